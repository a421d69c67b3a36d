// Internal interface of the warm-start network kernels (net_kernels.hip) used
// by the runner (net_api.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace lbmnet {

// A tensor view: element (n, c, y, x) is at p[n * bs + (c * H + y) * W + x].
struct View {
    void *p;
    int C, H, W;
    long long bs;
};

template <class TI, class TO>
hipError_t conv3x3(const View &in, const float *w, const float *bias, const View &out, int N, int cin, int cout,
                   bool relu, hipStream_t s);
// The same for bf16 input and output on matrix cores: the weights are first
// packed to bf16 [tap][cout][cin rounded up to 32] in wp (9 * cout * pad32(cin)
// values), then the convolution accumulates bf16 products in FP32.
int pad32(int c);
// The convolution on weights packed by pack_all (the network keeps its packed
// weights until the parameters change).
// pool (may be NULL): the 2 x 2 mean-pooled output ([C][H/2][W/2] per sample),
// written by the same launch where the layout allows (bf16 output, whole
// 8-pixel groups, 16-byte aligned planes, even H and W); *pooled (may be
// NULL) tells whether it was, otherwise the caller pools separately.  up,
// upped: the same for the nearest 2x upsampled output ([C][2H][2W]).
hipError_t conv3x3_mfma_packed(const View &in, const __bf16 *wp, const float *bias, const View &out, int N,
                               int cin, int cout, bool relu, hipStream_t s, const View *pool = nullptr,
                               bool *pooled = nullptr, const View *up = nullptr, bool *upped = nullptr);
// Packing jobs of one launch (k_pack_all): the weights of a 3x3 layer at
// theta + woff, [cout][cin][9] FP32, rounded to bf16 at base + out in the
// forward layout [t][co][pad32(cin)] (flip = 0, rows = cout, pad = pad32(cin))
// or flipped for the input gradient, [t][ci][pad32(cout)] with tap 8 - t
// (flip = 1, rows = cin, pad = pad32(cout)).
struct PackJob {
    int64_t woff, out;
    int32_t cin, cout, rows, pad, flip, unused;
};
struct PackJobs {
    static constexpr int MAX = 32;
    int32_t n, unused;
    PackJob job[MAX];
};
hipError_t pack_all(const float *theta, __bf16 *base, const PackJobs &jobs, hipStream_t s);
// The input gradient on weights packed (flipped) by pack_all.
hipError_t conv3x3_mfma_dx_packed(const View &dz, const __bf16 *wp, const View &dx, int N, int cin, int cout,
                                  hipStream_t s);
hipError_t flip_transpose(const float *w, float *wt, int cin, int cout, hipStream_t s);
int dw_chunks(int N, int H, int W, int cin, int cout);
// The weight gradient on matrix cores (bf16 activations x, the layer gradient
// dz already rounded to bf16), and its chunk count (partials hold chunks *
// cout * cin * 9 floats).  Both weight-gradient launchers also finish the
// layer's bias gradient, db[c] = sum of the nb partial sums bpart[c * nb ...]
// that relu_mask_bias left (skipped when bpart is NULL).
int dw_chunks_mfma(int N, int H, int W, int cin, int cout);
hipError_t conv3x3_dw_mfma(const View &x, const __bf16 *dz, int N, int cin, int cout, float *partial, int chunks,
                           float *dw, const float *bpart, int nb, float *db, hipStream_t s);
template <class TI>
hipError_t conv3x3_dw(const View &x, const float *dz, int N, int cin, int cout, float *partial, int chunks,
                      float *dw, const float *bpart, int nb, float *db, hipStream_t s);
// Layer gradient through the ReLU, dz = g * (y > 0), written in FP32 (dz) and/or
// rounded to bf16 (dzh) (either may be NULL), and the first pass of the bias
// gradient: per-workgroup sums of dz in part (bias_scratch(N, C, H, W) floats
// at most), *nparts of them per channel, contiguous by channel.
size_t bias_scratch(int N, int C, int H, int W);
template <class TA>
// pool_g / up_g (may be NULL): the adjoint of a following 2 x 2 mean pooling
// (g += pool_g / 4 at the pooled pixel) or of a following nearest 2x
// upsampling (g = sum of the 2 x 2 block of up_g) of the layer's output,
// folded into the same pass where the layout allows (g then not written, and
// for up_g not read), else run on g first.
hipError_t relu_mask_bias(const View &g, const View &y, int N, int C, float *dz, __bf16 *dzh, float *part,
                          int *nparts, hipStream_t s, const View *pool_g = nullptr, const View *up_g = nullptr);
template <class TA>
hipError_t pool(const View &in, const View &out, int N, int C, hipStream_t s);
hipError_t pool_back_acc(const View &dy, const View &dx, int N, int C, hipStream_t s);
template <class TA>
hipError_t up(const View &in, const View &out, int N, int C, hipStream_t s);
hipError_t up_back(const View &dy, const View &dx, int N, int C, hipStream_t s);
template <class TA>
hipError_t conv1x1(const View &in, const float *w, const float *b, int N, int cin, int cout, float *out,
                   hipStream_t s);
hipError_t conv1x1_dx(const float *g, const float *w, int N, int cin, int cout, int HW, const View &dx,
                      hipStream_t s);
int conv1x1_dw_scratch(int cin, int cout);
template <class TA>
hipError_t conv1x1_dw(const View &x, const float *g, int N, int cin, int cout, float *part, float *dw, float *db,
                      hipStream_t s);
int loss_blocks();
hipError_t loss_and_grad(const float *y, const float *t, const uint8_t *mask, int N, int C, int HW, double *part,
                         double *stats, float *g, hipStream_t s);
hipError_t adam(float *th, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s);
hipError_t zero(float *p, size_t n, hipStream_t s);

}  // namespace lbmnet
