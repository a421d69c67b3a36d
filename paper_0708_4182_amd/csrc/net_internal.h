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
hipError_t conv3x3_mfma(const View &in, const float *w, const float *bias, const View &out, int N, int cin,
                        int cout, bool relu, __bf16 *wp, hipStream_t s);
// The two halves of conv3x3_mfma: packing alone, and the convolution on
// weights packed earlier (the network keeps its packed weights until the
// parameters change).
hipError_t pack_weights(const float *w, __bf16 *wp, int cin, int cout, hipStream_t s);
hipError_t conv3x3_mfma_packed(const View &in, const __bf16 *wp, const float *bias, const View &out, int N,
                               int cin, int cout, bool relu, hipStream_t s);
// Input gradient of a 3x3 layer on matrix cores: dz is the layer gradient
// already rounded to bf16, the weights are rounded to bf16 as they are packed;
// wp holds 9 * cin * pad32(cout) bf16.
hipError_t conv3x3_mfma_dx(const View &dz, const float *w, const View &dx, int N, int cin, int cout, __bf16 *wp,
                           hipStream_t s);
hipError_t flip_transpose(const float *w, float *wt, int cin, int cout, hipStream_t s);
int dw_chunks(int N, int H, int W, int cin, int cout);
// The weight gradient on matrix cores (bf16 activations x, the layer gradient
// dz already rounded to bf16), and its chunk count (partials hold chunks *
// cout * cin * 9 floats).
int dw_chunks_mfma(int N, int H, int W, int cin, int cout);
hipError_t conv3x3_dw_mfma(const View &x, const __bf16 *dz, int N, int cin, int cout, float *partial, int chunks,
                           float *dw, hipStream_t s);
template <class TI>
hipError_t conv3x3_dw(const View &x, const float *dz, int N, int cin, int cout, float *partial, int chunks,
                      float *dw, hipStream_t s);
// floats of scratch bias_grad needs for C channels
int bias_scratch(int C);
hipError_t bias_grad(const float *dz, int N, int C, int HW, float *part, float *db, hipStream_t s);
template <class TA>
hipError_t relu_mask(const View &g, const View &y, int N, int C, float *dz, __bf16 *dzh, hipStream_t s);
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
