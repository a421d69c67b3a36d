// Runner of the warm-start network: the C ABI declared in include/lbm_net.h.
//
// Holds the layer plan of the 4-level encoder-decoder, carves every buffer
// (activations, concatenation buffers, gradients, parameters, Adam moments,
// scratch) out of the caller's device workspace, and issues the kernels of
// net_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_net.h"
#include "net_internal.h"

using lbmnet::View;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
thread_local std::string g_net_error;

// Layer order of the parameter vector (W[cout][cin][k][k] then b[cout]).
enum { E1A, E1B, E2A, E2B, E3A, E3B, BA, BB, D3A, D3B, D2A, D2B, D1A, D1B, OUT, NLAYERS };

struct Plan {
    int H, W, B, cin, cout, c[4];
    bool bf16;
    size_t asz;                      // bytes per activation element
    int lcin[NLAYERS], lcout[NLAYERS], lk[NLAYERS];
    size_t woff[NLAYERS], boff[NLAYERS];
    size_t nparams;
};

bool make_plan(const lbm_net_config *cfg, Plan &P, std::string &why) {
    if (!cfg) { why = "config is NULL"; return false; }
    if (cfg->H < 8 || cfg->W < 8 || cfg->H % 8 || cfg->W % 8) { why = "H and W must be multiples of 8"; return false; }
    if (cfg->batch < 1 || cfg->cin < 1 || cfg->cout < 1) { why = "batch, cin and cout must be >= 1"; return false; }
    // grid dimensions y and z (at most 65535) carry samples x channel blocks
    if (cfg->batch > 512) { why = "batch must be <= 512"; return false; }
    if (cfg->cin > 2048 || cfg->cout > 2048) { why = "cin and cout must be <= 2048"; return false; }
    for (int i = 0; i < 4; ++i)
        if (cfg->chans[i] < 1 || cfg->chans[i] > 2048) { why = "channel counts must be in [1, 2048]"; return false; }
    P.H = cfg->H; P.W = cfg->W; P.B = cfg->batch; P.cin = cfg->cin; P.cout = cfg->cout;
    for (int i = 0; i < 4; ++i) P.c[i] = cfg->chans[i];
    P.bf16 = cfg->act_bf16 != 0;
    P.asz = P.bf16 ? 2 : 4;
    const int c1 = P.c[0], c2 = P.c[1], c3 = P.c[2], c4 = P.c[3];
    const int spec[NLAYERS][3] = {{P.cin, c1, 3}, {c1, c1, 3}, {c1, c2, 3}, {c2, c2, 3}, {c2, c3, 3},
                                  {c3, c3, 3},    {c3, c4, 3}, {c4, c4, 3}, {c4 + c3, c3, 3}, {c3, c3, 3},
                                  {c3 + c2, c2, 3}, {c2, c2, 3}, {c2 + c1, c1, 3}, {c1, c1, 3}, {c1, P.cout, 1}};
    size_t o = 0;
    for (int l = 0; l < NLAYERS; ++l) {
        P.lcin[l] = spec[l][0]; P.lcout[l] = spec[l][1]; P.lk[l] = spec[l][2];
        P.woff[l] = o;
        o += (size_t)P.lcout[l] * P.lcin[l] * P.lk[l] * P.lk[l];
        P.boff[l] = o;
        o += P.lcout[l];
    }
    P.nparams = o;
    // the 3x3 convolutions index within one sample with 32-bit offsets
    int widest = 0;
    for (int l = 0; l < NLAYERS; ++l) widest = std::max(widest, std::max(P.lcin[l], P.lcout[l]));
    if ((int64_t)widest * P.H * P.W >= ((int64_t)1 << 31)) {
        why = "the widest layer of one sample must hold fewer than 2^31 values";
        return false;
    }
    return true;
}

// Named device buffers, laid out in one workspace.
struct Buffers {
    // activations (bf16 or fp32)
    char *e1a, *cat1, *p1, *e2a, *cat2, *p2, *e3a, *cat3, *p3, *ba, *bb, *d3a, *d3b, *d2a, *d2b, *d1a, *d1b;
    // gradients (fp32), same shapes
    float *g_e1a, *g_cat1, *g_p1, *g_e2a, *g_cat2, *g_p2, *g_e3a, *g_cat3, *g_p3, *g_ba, *g_bb, *g_d3a, *g_d3b,
        *g_d2a, *g_d2b, *g_d1a, *g_d1b, *g_out, *y, *dz, *wt, *partial;
    float *theta, *grad, *m, *v;
    __bf16 *wpf;                     // packed bf16 weights of every matrix-core layer: forward
    size_t wpoff[NLAYERS];           // layout of layer l at wpf + wpoff[l], flipped (input
    size_t wpboff[NLAYERS];          // gradient) at wpf + wpboff[l]
    __bf16 *dzh;                     // the layer gradient rounded to bf16 (bf16 build, input gradient)
    double *loss_part, *loss_stats;
    float *bpart;                    // per-workgroup partial sums of a layer's bias gradient
    size_t total, partial_floats, bpart_floats;
};

bool layout(const Plan &P, char *base, Buffers &b) {
    size_t off = 0;
    const size_t B = P.B, H = P.H, W = P.W;
    const int c1 = P.c[0], c2 = P.c[1], c3 = P.c[2], c4 = P.c[3];
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes, kAlign);
        return p;
    };
    auto act = [&](size_t C, size_t h, size_t w) { return take(B * C * h * w * P.asz); };
    auto grd = [&](size_t C, size_t h, size_t w) { return (float *)take(B * C * h * w * 4); };
    const size_t H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4, H8 = H / 8, W8 = W / 8;
    b.e1a = act(c1, H, W); b.cat1 = act(c2 + c1, H, W); b.p1 = act(c1, H2, W2); b.e2a = act(c2, H2, W2);
    b.cat2 = act(c3 + c2, H2, W2); b.p2 = act(c2, H4, W4); b.e3a = act(c3, H4, W4); b.cat3 = act(c4 + c3, H4, W4);
    b.p3 = act(c3, H8, W8); b.ba = act(c4, H8, W8); b.bb = act(c4, H8, W8); b.d3a = act(c3, H4, W4);
    b.d3b = act(c3, H4, W4); b.d2a = act(c2, H2, W2); b.d2b = act(c2, H2, W2); b.d1a = act(c1, H, W);
    b.d1b = act(c1, H, W);
    b.g_e1a = grd(c1, H, W); b.g_cat1 = grd(c2 + c1, H, W); b.g_p1 = grd(c1, H2, W2); b.g_e2a = grd(c2, H2, W2);
    b.g_cat2 = grd(c3 + c2, H2, W2); b.g_p2 = grd(c2, H4, W4); b.g_e3a = grd(c3, H4, W4);
    b.g_cat3 = grd(c4 + c3, H4, W4); b.g_p3 = grd(c3, H8, W8); b.g_ba = grd(c4, H8, W8); b.g_bb = grd(c4, H8, W8);
    b.g_d3a = grd(c3, H4, W4); b.g_d3b = grd(c3, H4, W4); b.g_d2a = grd(c2, H2, W2); b.g_d2b = grd(c2, H2, W2);
    b.g_d1a = grd(c1, H, W); b.g_d1b = grd(c1, H, W); b.g_out = grd(P.cout, H, W); b.y = grd(P.cout, H, W);
    // scratch: the largest layer output (dz) and transposed weights
    size_t dzmax = 0, wtmax = 0, partmax = 0, bpartmax = 0;
    const int lh[NLAYERS] = {(int)H, (int)H, (int)H2, (int)H2, (int)H4, (int)H4, (int)H8, (int)H8,
                             (int)H4, (int)H4, (int)H2, (int)H2, (int)H, (int)H, (int)H};
    const int lw[NLAYERS] = {(int)W, (int)W, (int)W2, (int)W2, (int)W4, (int)W4, (int)W8, (int)W8,
                             (int)W4, (int)W4, (int)W2, (int)W2, (int)W, (int)W, (int)W};
    for (int l = 0; l < NLAYERS; ++l) {
        dzmax = std::max(dzmax, B * P.lcout[l] * (size_t)lh[l] * lw[l]);
        wtmax = std::max(wtmax, (size_t)P.lcout[l] * P.lcin[l] * 9);
        if (P.lk[l] == 3) {
            const int ch = std::max(lbmnet::dw_chunks(P.B, lh[l], lw[l], P.lcin[l], P.lcout[l]),
                                    lbmnet::dw_chunks_mfma(P.B, lh[l], lw[l], P.lcin[l], P.lcout[l]));
            partmax = std::max(partmax, (size_t)ch * P.lcout[l] * P.lcin[l] * 9);
            bpartmax = std::max(bpartmax, lbmnet::bias_scratch(P.B, P.lcout[l], lh[l], lw[l]));
        } else {
            partmax = std::max(partmax, (size_t)lbmnet::conv1x1_dw_scratch(P.lcin[l], P.lcout[l]));
        }
    }
    size_t wpf = 0;
    for (int l = 0; l < NLAYERS; ++l) {
        b.wpoff[l] = wpf;
        if (l > 0 && P.lk[l] == 3) wpf += (size_t)9 * P.lcout[l] * lbmnet::pad32(P.lcin[l]);
    }
    for (int l = 0; l < NLAYERS; ++l) {
        b.wpboff[l] = wpf;
        if (l > 0 && P.lk[l] == 3) wpf += (size_t)9 * P.lcin[l] * lbmnet::pad32(P.lcout[l]);
    }
    b.wpf = (__bf16 *)take(2 * wpf);
    b.dz = (float *)take(4 * dzmax);
    b.dzh = (__bf16 *)take(2 * dzmax);
    b.wt = (float *)take(4 * wtmax);
    b.partial = (float *)take(4 * partmax);
    b.partial_floats = partmax;
    b.bpart = (float *)take(4 * bpartmax);
    b.bpart_floats = bpartmax;
    b.theta = (float *)take(4 * P.nparams);
    b.grad = (float *)take(4 * P.nparams);
    b.m = (float *)take(4 * P.nparams);
    b.v = (float *)take(4 * P.nparams);
    b.loss_part = (double *)take(16 * (size_t)lbmnet::loss_blocks());
    b.loss_stats = (double *)take(16);
    b.total = off;
    return true;
}

}  // namespace

struct lbm_net {
    Plan P;
    Buffers b;
    hipStream_t s = nullptr;
    int device = 0;
    int64_t adam_t = 0;
    bool have_grad = false;
    bool packed = false;             // b.wpf holds the current parameters in the forward layout
    bool packed_back = false;        // ... and in the flipped layout of the input gradient
    std::string err;
};

namespace {

lbm_status nfail(lbm_net *n, lbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    (n ? n->err : g_net_error) = buf;
    return st;
}

#define NHIP(n, expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return nfail((n), LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

View view(void *p, int C, int H, int W, int Cbuf, int c0, size_t esz) {
    View v;
    v.p = (char *)p + (size_t)c0 * H * W * esz;
    v.C = C;
    v.H = H;
    v.W = W;
    v.bs = (long long)Cbuf * H * W;
    return v;
}

// All tensors of one network pass.
struct Tensors {
    View x, e1a, e1, p1, e2a, e2, p2, e3a, e3, p3, ba, bb, up3, cat3, d3a, d3b, up2, cat2, d2a, d2b, up1, cat1,
        d1a, d1b;
    View g_e1a, g_e1, g_p1, g_e2a, g_e2, g_p2, g_e3a, g_e3, g_p3, g_ba, g_bb, g_up3, g_cat3, g_d3a, g_d3b, g_up2,
        g_cat2, g_d2a, g_d2b, g_up1, g_cat1, g_d1a, g_d1b;
};

Tensors tensors(const lbm_net *n, const float *x) {
    const Plan &P = n->P;
    const Buffers &b = n->b;
    const int H = P.H, W = P.W, H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4, H8 = H / 8, W8 = W / 8;
    const int c1 = P.c[0], c2 = P.c[1], c3 = P.c[2], c4 = P.c[3];
    const size_t a = P.asz;
    Tensors t;
    t.x = view((void *)x, P.cin, H, W, P.cin, 0, 4);
    t.e1a = view(b.e1a, c1, H, W, c1, 0, a);
    t.cat1 = view(b.cat1, c2 + c1, H, W, c2 + c1, 0, a);
    t.up1 = view(b.cat1, c2, H, W, c2 + c1, 0, a);
    t.e1 = view(b.cat1, c1, H, W, c2 + c1, c2, a);
    t.p1 = view(b.p1, c1, H2, W2, c1, 0, a);
    t.e2a = view(b.e2a, c2, H2, W2, c2, 0, a);
    t.cat2 = view(b.cat2, c3 + c2, H2, W2, c3 + c2, 0, a);
    t.up2 = view(b.cat2, c3, H2, W2, c3 + c2, 0, a);
    t.e2 = view(b.cat2, c2, H2, W2, c3 + c2, c3, a);
    t.p2 = view(b.p2, c2, H4, W4, c2, 0, a);
    t.e3a = view(b.e3a, c3, H4, W4, c3, 0, a);
    t.cat3 = view(b.cat3, c4 + c3, H4, W4, c4 + c3, 0, a);
    t.up3 = view(b.cat3, c4, H4, W4, c4 + c3, 0, a);
    t.e3 = view(b.cat3, c3, H4, W4, c4 + c3, c4, a);
    t.p3 = view(b.p3, c3, H8, W8, c3, 0, a);
    t.ba = view(b.ba, c4, H8, W8, c4, 0, a);
    t.bb = view(b.bb, c4, H8, W8, c4, 0, a);
    t.d3a = view(b.d3a, c3, H4, W4, c3, 0, a);
    t.d3b = view(b.d3b, c3, H4, W4, c3, 0, a);
    t.d2a = view(b.d2a, c2, H2, W2, c2, 0, a);
    t.d2b = view(b.d2b, c2, H2, W2, c2, 0, a);
    t.d1a = view(b.d1a, c1, H, W, c1, 0, a);
    t.d1b = view(b.d1b, c1, H, W, c1, 0, a);
    t.g_e1a = view(b.g_e1a, c1, H, W, c1, 0, 4);
    t.g_cat1 = view(b.g_cat1, c2 + c1, H, W, c2 + c1, 0, 4);
    t.g_up1 = view(b.g_cat1, c2, H, W, c2 + c1, 0, 4);
    t.g_e1 = view(b.g_cat1, c1, H, W, c2 + c1, c2, 4);
    t.g_p1 = view(b.g_p1, c1, H2, W2, c1, 0, 4);
    t.g_e2a = view(b.g_e2a, c2, H2, W2, c2, 0, 4);
    t.g_cat2 = view(b.g_cat2, c3 + c2, H2, W2, c3 + c2, 0, 4);
    t.g_up2 = view(b.g_cat2, c3, H2, W2, c3 + c2, 0, 4);
    t.g_e2 = view(b.g_cat2, c2, H2, W2, c3 + c2, c3, 4);
    t.g_p2 = view(b.g_p2, c2, H4, W4, c2, 0, 4);
    t.g_e3a = view(b.g_e3a, c3, H4, W4, c3, 0, 4);
    t.g_cat3 = view(b.g_cat3, c4 + c3, H4, W4, c4 + c3, 0, 4);
    t.g_up3 = view(b.g_cat3, c4, H4, W4, c4 + c3, 0, 4);
    t.g_e3 = view(b.g_cat3, c3, H4, W4, c4 + c3, c4, 4);
    t.g_p3 = view(b.g_p3, c3, H8, W8, c3, 0, 4);
    t.g_ba = view(b.g_ba, c4, H8, W8, c4, 0, 4);
    t.g_bb = view(b.g_bb, c4, H8, W8, c4, 0, 4);
    t.g_d3a = view(b.g_d3a, c3, H4, W4, c3, 0, 4);
    t.g_d3b = view(b.g_d3b, c3, H4, W4, c3, 0, 4);
    t.g_d2a = view(b.g_d2a, c2, H2, W2, c2, 0, 4);
    t.g_d2b = view(b.g_d2b, c2, H2, W2, c2, 0, 4);
    t.g_d1a = view(b.g_d1a, c1, H, W, c1, 0, 4);
    t.g_d1b = view(b.g_d1b, c1, H, W, c1, 0, 4);
    return t;
}

// Input, output and gradient views of each 3x3 layer.
struct LayerIO {
    View X, Y, gX, gY;
    bool has_gx;
};

void layer_io(const Tensors &t, LayerIO io[NLAYERS]) {
    io[E1A] = {t.x, t.e1a, View{}, t.g_e1a, false};
    io[E1B] = {t.e1a, t.e1, t.g_e1a, t.g_e1, true};
    io[E2A] = {t.p1, t.e2a, t.g_p1, t.g_e2a, true};
    io[E2B] = {t.e2a, t.e2, t.g_e2a, t.g_e2, true};
    io[E3A] = {t.p2, t.e3a, t.g_p2, t.g_e3a, true};
    io[E3B] = {t.e3a, t.e3, t.g_e3a, t.g_e3, true};
    io[BA] = {t.p3, t.ba, t.g_p3, t.g_ba, true};
    io[BB] = {t.ba, t.bb, t.g_ba, t.g_bb, true};
    io[D3A] = {t.cat3, t.d3a, t.g_cat3, t.g_d3a, true};
    io[D3B] = {t.d3a, t.d3b, t.g_d3a, t.g_d3b, true};
    io[D2A] = {t.cat2, t.d2a, t.g_cat2, t.g_d2a, true};
    io[D2B] = {t.d2a, t.d2b, t.g_d2a, t.g_d2b, true};
    io[D1A] = {t.cat1, t.d1a, t.g_cat1, t.g_d1a, true};
    io[D1B] = {t.d1a, t.d1b, t.g_d1a, t.g_d1b, true};
}

// Forward convolution of layer l: the first layer reads the FP32 input with
// FP32 products; with bf16 activations every other layer runs on matrix
// cores (bf16 weights and activations, FP32 accumulation).
// pool, up (may be NULL): the 2 x 2 pooled and the 2x upsampled output,
// produced by the same launch where possible (*pooled, *upped), else by the
// caller.
template <class TA>
hipError_t conv_fwd(lbm_net *n, int l, const View &X, const View &Y, int N, bool first, const View *pool = nullptr,
                    bool *pooled = nullptr, const View *up = nullptr, bool *upped = nullptr) {
    const Plan &P = n->P;
    const float *w = n->b.theta + P.woff[l], *bias = n->b.theta + P.boff[l];
    if (pooled) *pooled = false;
    if (upped) *upped = false;
    if (first) return lbmnet::conv3x3<float, TA>(X, w, bias, Y, N, P.lcin[l], P.lcout[l], true, n->s);
    if constexpr (sizeof(TA) == 2)
        return lbmnet::conv3x3_mfma_packed(X, n->b.wpf + n->b.wpoff[l], bias, Y, N, P.lcin[l], P.lcout[l], true,
                                           n->s, pool, pooled, up, upped);
    else return lbmnet::conv3x3<TA, TA>(X, w, bias, Y, N, P.lcin[l], P.lcout[l], true, n->s);
}

// Pack the bf16 weights of every matrix-core layer in one launch: the forward
// layout, and with backward also the flipped one of the input gradients.
lbm_status pack(lbm_net *n, bool backward) {
    const Plan &P = n->P;
    lbmnet::PackJobs jobs{};
    for (int flip = 0; flip < (backward ? 2 : 1); ++flip)
        for (int l = 1; l < NLAYERS; ++l) {
            if (P.lk[l] != 3) continue;
            if (jobs.n >= lbmnet::PackJobs::MAX) return nfail(n, LBM_EINVAL, "too many packing jobs");
            lbmnet::PackJob &j = jobs.job[jobs.n++];
            j.woff = (int64_t)P.woff[l];
            j.out = (int64_t)(flip ? n->b.wpboff[l] : n->b.wpoff[l]);
            j.cin = P.lcin[l];
            j.cout = P.lcout[l];
            j.flip = flip;
            j.rows = flip ? P.lcin[l] : P.lcout[l];
            j.pad = lbmnet::pad32(flip ? P.lcout[l] : P.lcin[l]);
        }
    NHIP(n, lbmnet::pack_all(n->b.theta, n->b.wpf, jobs, n->s));
    n->packed = true;
    n->packed_back = backward;
    return LBM_OK;
}

template <class TA>
lbm_status forward_t(lbm_net *n, const float *x, float *y, int N) {
    const Plan &P = n->P;
    const Tensors t = tensors(n, x);
    LayerIO io[NLAYERS];
    layer_io(t, io);
    hipStream_t s = n->s;
    if (sizeof(TA) == 2 && !n->packed) {     // pack once per parameter update
        if (lbm_status st = pack(n, false)) return st;
    }
    bool pooled = false, upped = false;
    NHIP(n, (conv_fwd<TA>(n, E1A, io[E1A].X, io[E1A].Y, N, true)));
    NHIP(n, (conv_fwd<TA>(n, E1B, io[E1B].X, io[E1B].Y, N, false, &t.p1, &pooled)));
    if (!pooled) NHIP(n, lbmnet::pool<TA>(t.e1, t.p1, N, P.c[0], s));
    NHIP(n, (conv_fwd<TA>(n, E2A, io[E2A].X, io[E2A].Y, N, false)));
    NHIP(n, (conv_fwd<TA>(n, E2B, io[E2B].X, io[E2B].Y, N, false, &t.p2, &pooled)));
    if (!pooled) NHIP(n, lbmnet::pool<TA>(t.e2, t.p2, N, P.c[1], s));
    NHIP(n, (conv_fwd<TA>(n, E3A, io[E3A].X, io[E3A].Y, N, false)));
    NHIP(n, (conv_fwd<TA>(n, E3B, io[E3B].X, io[E3B].Y, N, false, &t.p3, &pooled)));
    if (!pooled) NHIP(n, lbmnet::pool<TA>(t.e3, t.p3, N, P.c[2], s));
    NHIP(n, (conv_fwd<TA>(n, BA, io[BA].X, io[BA].Y, N, false)));
    NHIP(n, (conv_fwd<TA>(n, BB, io[BB].X, io[BB].Y, N, false, nullptr, nullptr, &t.up3, &upped)));
    if (!upped) NHIP(n, lbmnet::up<TA>(t.bb, t.up3, N, P.c[3], s));
    NHIP(n, (conv_fwd<TA>(n, D3A, io[D3A].X, io[D3A].Y, N, false)));
    NHIP(n, (conv_fwd<TA>(n, D3B, io[D3B].X, io[D3B].Y, N, false, nullptr, nullptr, &t.up2, &upped)));
    if (!upped) NHIP(n, lbmnet::up<TA>(t.d3b, t.up2, N, P.c[2], s));
    NHIP(n, (conv_fwd<TA>(n, D2A, io[D2A].X, io[D2A].Y, N, false)));
    NHIP(n, (conv_fwd<TA>(n, D2B, io[D2B].X, io[D2B].Y, N, false, nullptr, nullptr, &t.up1, &upped)));
    if (!upped) NHIP(n, lbmnet::up<TA>(t.d2b, t.up1, N, P.c[1], s));
    NHIP(n, (conv_fwd<TA>(n, D1A, io[D1A].X, io[D1A].Y, N, false)));
    NHIP(n, (conv_fwd<TA>(n, D1B, io[D1B].X, io[D1B].Y, N, false)));
    NHIP(n, lbmnet::conv1x1<TA>(t.d1b, n->b.theta + P.woff[OUT], n->b.theta + P.boff[OUT], N, P.c[0], P.cout, y, s));
    return LBM_OK;
}

// Gradients of one conv3x3 layer from the gradient of its (post-ReLU) output.
// pool_g / up_g (may be NULL): the layer's output also feeds a 2 x 2 pooling
// with gradient pool_g, or only a 2x upsampling with gradient up_g; their
// adjoints run in the ReLU-mask pass (folded where the layout allows).
template <class TA>
lbm_status conv_back(lbm_net *n, int l, const LayerIO &io, int N, const View *pool_g = nullptr,
                     const View *up_g = nullptr) {
    const Plan &P = n->P;
    Buffers &b = n->b;
    const int cin = P.lcin[l], cout = P.lcout[l], H = io.Y.H, W = io.Y.W;
    const bool mfma = sizeof(TA) == 2 && l != E1A;   // bf16 build, bf16 input activations
    // dz in FP32 where an FP32 gradient kernel reads it, rounded to bf16 for the
    // matrix-core ones, and the bias gradient's per-workgroup sums, which the
    // weight-gradient launch finishes
    if (lbmnet::bias_scratch(N, cout, H, W) > b.bpart_floats) return nfail(n, LBM_EINVAL, "bias scratch too small");
    int nb = 0;
    NHIP(n, lbmnet::relu_mask_bias<TA>(io.gY, io.Y, N, cout, mfma ? nullptr : b.dz, sizeof(TA) == 2 ? b.dzh : nullptr,
                                       b.bpart, &nb, n->s, pool_g, up_g));
    float *db = b.grad + P.boff[l];
    const int chunks = mfma ? lbmnet::dw_chunks_mfma(N, H, W, cin, cout) : lbmnet::dw_chunks(N, H, W, cin, cout);
    if ((size_t)chunks * cout * cin * 9 > b.partial_floats) return nfail(n, LBM_EINVAL, "dW scratch too small");
    if (l == E1A)
        NHIP(n, lbmnet::conv3x3_dw<float>(io.X, b.dz, N, cin, cout, b.partial, chunks, b.grad + P.woff[l], b.bpart, nb,
                                          db, n->s));
    else if (mfma)
        NHIP(n, lbmnet::conv3x3_dw_mfma(io.X, b.dzh, N, cin, cout, b.partial, chunks, b.grad + P.woff[l], b.bpart, nb,
                                        db, n->s));
    else
        NHIP(n, lbmnet::conv3x3_dw<TA>(io.X, b.dz, N, cin, cout, b.partial, chunks, b.grad + P.woff[l], b.bpart, nb, db,
                                       n->s));
    if (io.has_gx) {
        const View dz = view(b.dz, cout, H, W, cout, 0, 4);
        if (sizeof(TA) == 2) {
            // bf16 build: matrix cores, dz (rounded to bf16 by relu_mask) and W rounded to bf16
            const View dzh = view(b.dzh, cout, H, W, cout, 0, 2);
            NHIP(n, lbmnet::conv3x3_mfma_dx_packed(dzh, b.wpf + b.wpboff[l], io.gX, N, cin, cout, n->s));
        } else {
            NHIP(n, lbmnet::flip_transpose(b.theta + P.woff[l], b.wt, cin, cout, n->s));
            NHIP(n, (lbmnet::conv3x3<float, float>(dz, b.wt, nullptr, io.gX, N, cout, cin, false, n->s)));
        }
    }
    return LBM_OK;
}

template <class TA>
lbm_status gradient_t(lbm_net *n, const float *x, const float *tgt, const uint8_t *fluid, int N) {
    const Plan &P = n->P;
    Buffers &b = n->b;
    hipStream_t s = n->s;
    lbm_status st;
    if (sizeof(TA) == 2 && !(n->packed && n->packed_back) && (st = pack(n, true))) return st;
    st = forward_t<TA>(n, x, b.y, N);
    if (st) return st;
    const int HW = P.H * P.W;
    NHIP(n, lbmnet::loss_and_grad(b.y, tgt, fluid, N, P.cout, HW, b.loss_part, b.loss_stats, b.g_out, s));
    const Tensors t = tensors(n, x);
    LayerIO io[NLAYERS];
    layer_io(t, io);
    NHIP(n, lbmnet::conv1x1_dw<TA>(t.d1b, b.g_out, N, P.c[0], P.cout, b.partial, b.grad + P.woff[OUT],
                                    b.grad + P.boff[OUT], s));
    NHIP(n, lbmnet::conv1x1_dx(b.g_out, b.theta + P.woff[OUT], N, P.c[0], P.cout, HW, t.g_d1b, s));
#define BACK(L, ...)                                                  \
    do {                                                              \
        if ((st = conv_back<TA>(n, L, io[L], N, ##__VA_ARGS__))) return st; \
    } while (0)
    BACK(D1B);
    BACK(D1A);
    BACK(D2B, nullptr, &t.g_up1);
    BACK(D2A);
    BACK(D3B, nullptr, &t.g_up2);
    BACK(D3A);
    BACK(BB, nullptr, &t.g_up3);
    BACK(BA);
    BACK(E3B, &t.g_p3);
    BACK(E3A);
    BACK(E2B, &t.g_p2);
    BACK(E2A);
    BACK(E1B, &t.g_p1);
    BACK(E1A);
#undef BACK
    n->have_grad = true;
    return LBM_OK;
}

lbm_status check_n(lbm_net *n, int32_t N) {
    if (!n) return LBM_EINVAL;
    if (N < 1 || N > n->P.B) return nfail(n, LBM_EINVAL, "n must be in [1, %d]", n->P.B);
    return LBM_OK;
}

}  // namespace

extern "C" {

int64_t lbm_net_param_count(const lbm_net_config *cfg) {
    Plan P;
    std::string why;
    return make_plan(cfg, P, why) ? (int64_t)P.nparams : -1;
}

size_t lbm_net_workspace_bytes(const lbm_net_config *cfg) {
    Plan P;
    std::string why;
    if (!make_plan(cfg, P, why)) return 0;
    Buffers b;
    layout(P, nullptr, b);
    return b.total;
}

lbm_status lbm_net_create(lbm_net **out, const lbm_net_config *cfg, void *ws, size_t bytes, void *stream) {
    if (!out) return nfail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    Plan P;
    std::string why;
    if (!make_plan(cfg, P, why)) return nfail(nullptr, LBM_EINVAL, "%s", why.c_str());
    Buffers b;
    layout(P, nullptr, b);
    if (!ws || (uintptr_t)ws % kAlign) return nfail(nullptr, LBM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (bytes < b.total) return nfail(nullptr, LBM_ENOMEM, "workspace has %zu bytes, %zu needed", bytes, b.total);
    lbm_net *n = new lbm_net();
    n->P = P;
    layout(P, (char *)ws, n->b);
    n->s = (hipStream_t)stream;
    if (hipGetDevice(&n->device) != hipSuccess) {
        delete n;
        return nfail(nullptr, LBM_EDEVICE, "hipGetDevice failed");
    }
    hipError_t e = hipSuccess;
    for (float *p : {n->b.theta, n->b.grad, n->b.m, n->b.v})
        if (e == hipSuccess) e = lbmnet::zero(p, P.nparams, n->s);
    if (e == hipSuccess) e = hipStreamSynchronize(n->s);
    if (e != hipSuccess) {
        delete n;
        return nfail(nullptr, LBM_EDEVICE, "workspace clear failed: %s", hipGetErrorString(e));
    }
    *out = n;
    return LBM_OK;
}

lbm_status lbm_net_set_params(lbm_net *n, const float *host, int64_t count) {
    if (!n || !host) return LBM_EINVAL;
    if (count != (int64_t)n->P.nparams) return nfail(n, LBM_EINVAL, "expected %zu parameters", n->P.nparams);
    n->packed = false;
    n->packed_back = false;
    NHIP(n, hipMemcpyAsync(n->b.theta, host, 4 * n->P.nparams, hipMemcpyHostToDevice, n->s));
    NHIP(n, lbmnet::zero(n->b.m, n->P.nparams, n->s));
    NHIP(n, lbmnet::zero(n->b.v, n->P.nparams, n->s));
    NHIP(n, hipStreamSynchronize(n->s));
    n->adam_t = 0;
    n->have_grad = false;
    return LBM_OK;
}

lbm_status lbm_net_get_params(lbm_net *n, float *host, int64_t count) {
    if (!n || !host) return LBM_EINVAL;
    if (count != (int64_t)n->P.nparams) return nfail(n, LBM_EINVAL, "expected %zu parameters", n->P.nparams);
    NHIP(n, hipMemcpyAsync(host, n->b.theta, 4 * n->P.nparams, hipMemcpyDeviceToHost, n->s));
    NHIP(n, hipStreamSynchronize(n->s));
    return LBM_OK;
}

lbm_status lbm_net_forward(lbm_net *n, const float *x, float *y, int32_t N) {
    lbm_status st = check_n(n, N);
    if (st) return st;
    if (!x || !y) return nfail(n, LBM_EINVAL, "x and y must not be NULL");
    return n->P.bf16 ? forward_t<__bf16>(n, x, y, N) : forward_t<float>(n, x, y, N);
}

lbm_status lbm_net_gradient(lbm_net *n, const float *x, const float *t, const uint8_t *fluid, int32_t N,
                            double *loss, float *grad_host) {
    lbm_status st = check_n(n, N);
    if (st) return st;
    if (!x || !t || !fluid) return nfail(n, LBM_EINVAL, "x, t and fluid must not be NULL");
    st = n->P.bf16 ? gradient_t<__bf16>(n, x, t, fluid, N) : gradient_t<float>(n, x, t, fluid, N);
    if (st) return st;
    double stats[2];
    NHIP(n, hipMemcpyAsync(stats, n->b.loss_stats, sizeof stats, hipMemcpyDeviceToHost, n->s));
    if (grad_host)
        NHIP(n, hipMemcpyAsync(grad_host, n->b.grad, 4 * n->P.nparams, hipMemcpyDeviceToHost, n->s));
    NHIP(n, hipStreamSynchronize(n->s));
    if (loss) *loss = stats[0];
    return LBM_OK;
}

lbm_status lbm_net_adam(lbm_net *n, float lr, float b1, float b2, float eps) {
    if (!n) return LBM_EINVAL;
    if (!n->have_grad) return nfail(n, LBM_ESTATE, "no gradient to apply");
    if (!(lr > 0.f && b1 >= 0.f && b1 < 1.f && b2 >= 0.f && b2 < 1.f && eps > 0.f) || !std::isfinite(lr))
        return nfail(n, LBM_EINVAL, "Adam needs lr > 0, 0 <= beta < 1, eps > 0");
    n->adam_t += 1;
    const double c1 = 1.0 - std::pow((double)b1, (double)n->adam_t);
    const double c2 = 1.0 - std::pow((double)b2, (double)n->adam_t);
    n->packed = false;
    n->packed_back = false;
    NHIP(n, lbmnet::adam(n->b.theta, n->b.grad, n->b.m, n->b.v, (int)n->P.nparams, lr, b1, b2, eps, (float)c1,
                         (float)c2, n->s));
    n->have_grad = false;
    return LBM_OK;
}

lbm_status lbm_net_train_step(lbm_net *n, const float *x, const float *t, const uint8_t *fluid, int32_t N,
                              float lr, double *loss) {
    lbm_status st = check_n(n, N);
    if (st) return st;
    if (!x || !t || !fluid) return nfail(n, LBM_EINVAL, "x, t and fluid must not be NULL");
    if (!(lr > 0.f) || !std::isfinite(lr)) return nfail(n, LBM_EINVAL, "lr must be positive and finite");
    st = n->P.bf16 ? gradient_t<__bf16>(n, x, t, fluid, N) : gradient_t<float>(n, x, t, fluid, N);
    if (st) return st;
    if ((st = lbm_net_adam(n, lr, 0.9f, 0.999f, 1e-8f))) return st;
    if (loss) {
        double stats[2];
        NHIP(n, hipMemcpyAsync(stats, n->b.loss_stats, sizeof stats, hipMemcpyDeviceToHost, n->s));
        NHIP(n, hipStreamSynchronize(n->s));
        *loss = stats[0];
    }
    return LBM_OK;
}

void lbm_net_free(lbm_net *n) { delete n; }

const char *lbm_net_last_error(const lbm_net *n) { return n ? n->err.c_str() : g_net_error.c_str(); }

}  // extern "C"
