// HIP kernels of the warm-start network (training and inference) for gfx950.
//
// Tensors are NCHW; activations are stored as bf16 (or fp32 for checking) and
// every product and sum is FP32.  A tensor view is a pointer to channel 0 of
// sample 0 plus the channel count, H, W and the distance between samples, so
// a channel slice of a concatenation buffer is a view like any other.
// Convolutions are 3x3, periodic along x and zero-padded along y (the
// channels are periodic in x and bounded by walls in y).
#include "net_internal.h"

#include <type_traits>

namespace lbmnet {
namespace {

template <class T> __device__ __forceinline__ float tof(T v) { return (float)v; }
template <class T> __device__ __forceinline__ T fromf(float v) { return (T)v; }

// --------------------------------------------------------------- conv 3x3
// One workgroup: 8 x 32 output pixels of one sample, 16 output channels.
// Input channels are staged through LDS 8 at a time, with a one-pixel halo
// (x wraps around, y outside the lattice reads 0).
constexpr int TH = 8, TW = 32, CO_T = 16, CI_T = 8;

template <class TI, class TO>
__global__ void __launch_bounds__(256) k_conv3x3(View in, const float *__restrict__ w,
                                                 const float *__restrict__ bias, View out, int cin,
                                                 int cout, int relu) {
    __shared__ float xs[CI_T][TH + 2][TW + 2];
    __shared__ float4 ws[CI_T][9][CO_T / 4];
    const int H = in.H, W = in.W;
    const int tiles_x = (W + TW - 1) / TW;
    const int tx0 = (blockIdx.x % tiles_x) * TW, ty0 = (blockIdx.x / tiles_x) * TH;
    const int ncob = (cout + CO_T - 1) / CO_T;
    const int n = blockIdx.y / ncob, co0 = (blockIdx.y % ncob) * CO_T;
    const int tid = threadIdx.x, px = tid % TW, py = tid / TW;
    const TI *__restrict__ xin = static_cast<const TI *>(in.p) + (size_t)n * in.bs;
    // biases read up front (a load in the epilogue would make each store wait)
    float bv[CO_T];
#pragma unroll
    for (int o = 0; o < CO_T; ++o) bv[o] = (bias != nullptr && co0 + o < cout) ? bias[co0 + o] : 0.f;
    float acc[CO_T];
#pragma unroll
    for (int o = 0; o < CO_T; ++o) acc[o] = 0.f;
    int ci0 = 0;
    do {       // cin >= 1
        // only the chunk's real channels are staged and summed (the first
        // layer has 3 input planes); many workgroups per CU hide the load
        // latency of this loop
        const int cn = min(CI_T, cin - ci0);
        for (int e = tid; e < cn * (TH + 2) * (TW + 2); e += 256) {
            const int c = e / ((TH + 2) * (TW + 2)), r = (e / (TW + 2)) % (TH + 2), q = e % (TW + 2);
            const int y = ty0 - 1 + r;
            int x = tx0 - 1 + q;       // periodic
            if (x < 0) x += W;
            if (x >= W) x -= W;
            if (x >= W) x %= W;        // lattices narrower than a tile
            float v = 0.f;
            if (y >= 0 && y < H) v = tof(xin[(size_t)(ci0 + c) * H * W + (size_t)y * W + x]);
            xs[c][r][q] = v;
        }
        for (int e = tid; e < cn * 9 * CO_T; e += 256) {
            const int c = e / (9 * CO_T), t = (e / CO_T) % 9, o = e % CO_T;
            float v = 0.f;
            if (co0 + o < cout) v = w[((size_t)(co0 + o) * cin + ci0 + c) * 9 + t];
            reinterpret_cast<float *>(&ws[c][t][0])[o] = v;
        }
        __syncthreads();
#pragma unroll 2
        for (int c = 0; c < cn; ++c) {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const float xc = xs[c][py + t / 3][px + t % 3];
#pragma unroll
                for (int o4 = 0; o4 < CO_T / 4; ++o4) {
                    const float4 wq = ws[c][t][o4];
                    acc[4 * o4 + 0] += wq.x * xc;
                    acc[4 * o4 + 1] += wq.y * xc;
                    acc[4 * o4 + 2] += wq.z * xc;
                    acc[4 * o4 + 3] += wq.w * xc;
                }
            }
        }
        __syncthreads();
        ci0 += CI_T;
    } while (ci0 < cin);
    const int y = ty0 + py, x = tx0 + px;
    if (y >= H || x >= W) return;
    TO *__restrict__ yo = static_cast<TO *>(out.p) + (size_t)n * out.bs;
#pragma unroll
    for (int o = 0; o < CO_T; ++o) {
        if (co0 + o >= cout) break;
        float v = acc[o] + bv[o];
        if (relu) v = fmaxf(v, 0.f);
        yo[(size_t)(co0 + o) * H * W + (size_t)y * W + x] = fromf<TO>(v);
    }
}

// W'[ci][co][8 - t] = W[co][ci][t]: the weights of the transposed convolution
// used for the input gradient.
__global__ void k_flip_transpose(const float *__restrict__ w, float *__restrict__ wt, int cin, int cout) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cin * cout * 9) return;
    const int t = i % 9, co = (i / 9) % cout, ci = i / (9 * cout);
    wt[i] = w[((size_t)co * cin + ci) * 9 + (8 - t)];
}

// ------------------------------------------------------- weight gradient
// dW[co][ci][t] = sum over samples and pixels of dz[co](p) x[ci](p + shift t).
// Workgroup (chunk, co block of CO_B, ci block of CI_B) accumulates over the
// tiles of its chunk; thread t owns (co, ci) = ((t / CI_B) % CO_B, t % CI_B),
// all 9 taps and the output rows of part t / (CO_B CI_B) of PS parts of the
// tile.  For each output row it walks the three staged input rows with a
// sliding window of 3 values, so one dz read and three x reads feed 9 FMAs.
// Channel strides in LDS are odd, so the ci (and co) of a wave hit distinct
// banks.  The PS row parts are added in order at the end.  Partials
// [chunk][co][ci][tap] are summed in chunk order by k_sum_grads.  16 x 16 x 1
// in general; 32 x 4 x 2 for the first layer (three input planes), which
// would leave 13 of 16 threads idle in the general shape.
constexpr int XS_STRIDE = (TH + 2) * (TW + 2) + 1, DS_STRIDE = TH * TW + 1;

template <class TI, int CO_B, int CI_B, int PS>
__global__ void __launch_bounds__(256) k_conv3x3_dw(View x, const float *__restrict__ dz, int N, int cin,
                                                    int cout, int tiles_per_chunk,
                                                    float *__restrict__ partial) {
    static_assert(CO_B * CI_B * PS == 256 && TH % PS == 0, "thread mapping");
    static_assert((PS - 1) * 9 * CO_B * CI_B <= CO_B * DS_STRIDE, "row-part sums fit in the dz stage");
    constexpr int DW_CO = CO_B, DW_CI = CI_B, ROWS = TH / PS;
    __shared__ float xs[DW_CI * XS_STRIDE];
    __shared__ float ds[DW_CO * DS_STRIDE];
    const int H = x.H, W = x.W;
    const int tiles_x = (W + TW - 1) / TW, tiles_y = (H + TH - 1) / TH;
    const int ntiles = N * tiles_x * tiles_y;
    const int chunk = blockIdx.x, co0 = blockIdx.y * DW_CO, ci0 = blockIdx.z * DW_CI;
    const int tid = threadIdx.x;
    const int my_co = (tid / DW_CI) % DW_CO, my_ci = tid % DW_CI, part = tid / (DW_CO * DW_CI);
    float acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.f;
    const int t_begin = chunk * tiles_per_chunk, t_end = min(ntiles, t_begin + tiles_per_chunk);
    for (int tile = t_begin; tile < t_end; ++tile) {
        const int n = tile / (tiles_x * tiles_y), rem = tile % (tiles_x * tiles_y);
        const int ty0 = (rem / tiles_x) * TH, tx0 = (rem % tiles_x) * TW;
        const TI *__restrict__ xin = static_cast<const TI *>(x.p) + (size_t)n * x.bs;
        for (int e = tid; e < DW_CI * (TH + 2) * (TW + 2); e += 256) {
            const int c = e / ((TH + 2) * (TW + 2)), r = (e / (TW + 2)) % (TH + 2), q = e % (TW + 2);
            const int y = ty0 - 1 + r;
            const int xx = (tx0 - 1 + q + W) % W;
            float v = 0.f;
            if (ci0 + c < cin && y >= 0 && y < H) v = tof(xin[(size_t)(ci0 + c) * H * W + (size_t)y * W + xx]);
            xs[c * XS_STRIDE + r * (TW + 2) + q] = v;
        }
        for (int e = tid; e < DW_CO * TH * TW; e += 256) {
            const int o = e / (TH * TW), p = e % (TH * TW);
            const int y = ty0 + p / TW, xx = tx0 + p % TW;
            float v = 0.f;
            if (co0 + o < cout && y < H && xx < W)
                v = dz[((size_t)n * cout + co0 + o) * H * W + (size_t)y * W + xx];
            ds[o * DS_STRIDE + p] = v;
        }
        __syncthreads();
        const float *__restrict__ xc = xs + my_ci * XS_STRIDE;
        const float *__restrict__ dc = ds + my_co * DS_STRIDE;
        for (int py = part * ROWS; py < (part + 1) * ROWS; ++py) {
            const float *r0 = xc + py * (TW + 2), *r1 = r0 + (TW + 2), *r2 = r1 + (TW + 2);
            float a0 = r0[0], a1 = r0[1], b0 = r1[0], b1 = r1[1], c0 = r2[0], c1 = r2[1];
#pragma unroll 8
            for (int px = 0; px < TW; ++px) {
                const float d = dc[py * TW + px];
                const float a2 = r0[px + 2], b2 = r1[px + 2], c2 = r2[px + 2];
                acc[0] += d * a0; acc[1] += d * a1; acc[2] += d * a2;
                acc[3] += d * b0; acc[4] += d * b1; acc[5] += d * b2;
                acc[6] += d * c0; acc[7] += d * c1; acc[8] += d * c2;
                a0 = a1; a1 = a2; b0 = b1; b1 = b2; c0 = c1; c1 = c2;
            }
        }
        __syncthreads();
    }
    if constexpr (PS > 1) {
        constexpr int Q = DW_CO * DW_CI;
        const int q = tid % Q;
        if (part > 0)
#pragma unroll
            for (int t = 0; t < 9; ++t) ds[((part - 1) * 9 + t) * Q + q] = acc[t];
        __syncthreads();
        if (part > 0) return;
        for (int k = 1; k < PS; ++k)
#pragma unroll
            for (int t = 0; t < 9; ++t) acc[t] += ds[((k - 1) * 9 + t) * Q + q];
    }
    if (ci0 + my_ci >= cin || co0 + my_co >= cout) return;
    float *__restrict__ dst = partial + (((size_t)chunk * cout + co0 + my_co) * cin + ci0 + my_ci) * 9;
#pragma unroll
    for (int t = 0; t < 9; ++t) dst[t] = acc[t];
}

// The two gradient sums of a 3x3 layer in one launch, each in a fixed order:
// dw[i] = sum over k < nchunks of partial[k n + i] (i < n), and, in the
// workgroups after the first wblocks, db[c] = sum over k < nb of
// bpart[c nb + k] (c < C; skipped when bpart is NULL).  A workgroup covers OB
// outputs with G = 256 / OB threads each: thread (o, g) adds the terms k = g,
// g + G, ... in eight running sums (eight loads in flight), those are added in
// a fixed tree, then the G thread sums in order of g.
template <int OB>
__global__ void __launch_bounds__(256) k_sum_grads(const float *__restrict__ partial, int nchunks, int n,
                                                   float *__restrict__ dw, const float *__restrict__ bpart, int nb,
                                                   int C, float *__restrict__ db, int wblocks) {
    constexpr int G = 256 / OB;
    __shared__ float sh[256];
    const int o = threadIdx.x % OB, g = threadIdx.x / OB;
    const bool bias = (int)blockIdx.x >= wblocks;
    const int i = (bias ? (int)blockIdx.x - wblocks : (int)blockIdx.x) * OB + o;
    const int count = bias ? nb : nchunks;
    const bool live = bias ? i < C : i < n;
    // term k of output i
    const float *base = bias ? bpart + (size_t)i * nb : partial + i;
    const size_t step = bias ? 1 : (size_t)n;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (live) {
        int k = g;
        for (; k + 7 * G < count; k += 8 * G) {
#pragma unroll
            for (int j = 0; j < 8; ++j) s[j] += base[(size_t)(k + j * G) * step];
        }
#pragma unroll
        for (int j = 0; j < 7; ++j)
            if (k + j * G < count) s[j] += base[(size_t)(k + j * G) * step];
    }
    sh[threadIdx.x] = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
    __syncthreads();
    if (g != 0 || !live) return;
    float t = sh[o];
    for (int q = 1; q < G; ++q) t += sh[q * OB + o];
    if (bias) db[i] = t;
    else dw[i] = t;
}

// Sum of v over the workgroup (256 threads), the same tree on every run: a
// butterfly within each wave, then the four wave sums in order.  Every thread
// of the workgroup must call it.
__device__ __forceinline__ float wg_sum256(float v, float *sh4) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) sh4[threadIdx.x >> 6] = v;
    __syncthreads();
    return (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
}

// Layer gradient through the ReLU, dz = g * (y > 0) (the derivative from the
// stored output), with the bias gradient's first pass folded in: workgroup
// (b, c, n) covers a block of pixels of plane (n, c) and writes the sum of its
// dz values to part[(c * N + n) * gridDim.x + b]; k_sum_grads adds those in
// a fixed order.  dz is written in FP32 (dz, when non-null: the FP32 weight
// and input gradients) and rounded to bf16 (dzh, when non-null: the matrix-
// core gradients).  Grids are (pixel blocks, channel, sample), so a thread
// finds its element without 64-bit divisions.
template <class TA>
__global__ void __launch_bounds__(256) k_relu_mask(View g, View y, int N, int C, float *__restrict__ dz,
                                                   __bf16 *__restrict__ dzh, float *__restrict__ part) {
    __shared__ float sh4[4];
    const uint32_t HW = (uint32_t)y.H * (uint32_t)y.W;
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t c = blockIdx.y, n = blockIdx.z;
    float v = 0.f;
    if (p < HW) {
        const size_t r = (size_t)c * HW + p, i = ((size_t)n * C + c) * HW + p;
        const float gv = static_cast<const float *>(g.p)[n * g.bs + r];
        const float yv = tof(static_cast<const TA *>(y.p)[n * y.bs + r]);
        v = yv > 0.f ? gv : 0.f;
        if (dz) dz[i] = v;
        if (dzh) dzh[i] = (__bf16)v;
    }
    const float t = wg_sum256(v, sh4);
    if (threadIdx.x == 0) part[((size_t)c * N + n) * gridDim.x + blockIdx.x] = t;
}

// The same, four pixels per thread (HW % 4 == 0 and aligned planes): 16-byte
// FP32 and 8-byte bf16 accesses.
//
// The layer's output gradient g itself may be given in one of two other
// forms, so that the adjoint passes of pooling and upsampling are not needed:
// pg.p != NULL: g plus a quarter of the gradient pg of its 2 x 2 mean pooling
// (H / 2 x W / 2 planes), as the pooling adjoint would accumulate it;
// ug.p != NULL: g is the sum over each 2 x 2 block of ug, the gradient of its
// nearest 2x upsampling (2H x 2W planes), and g.p is not read.  Both in the
// operand order of the adjoint kernels.
template <class TA>
__global__ void __launch_bounds__(256) k_relu_mask4(View g, View y, int N, int C, float *__restrict__ dz,
                                                    __bf16 *__restrict__ dzh, float *__restrict__ part, View pg,
                                                    View ug) {
    __shared__ float sh4[4];
    const uint32_t HW = (uint32_t)y.H * (uint32_t)y.W;
    const uint32_t p = 4u * (blockIdx.x * blockDim.x + threadIdx.x);
    const uint32_t c = blockIdx.y, n = blockIdx.z;
    float sum = 0.f;
    if (p < HW) {
        const size_t r = (size_t)c * HW + p, i = ((size_t)n * C + c) * HW + p;
        float4 gv;
        const uint32_t W = (uint32_t)y.W, yy = p / W, xx = p - yy * W;   // four pixels of one row
        if (ug.p != nullptr) {
            const float *u = static_cast<const float *>(ug.p) + n * ug.bs + (size_t)c * ug.H * ug.W +
                             (size_t)(2 * yy) * ug.W + 2 * xx;
            const float4 a0 = *reinterpret_cast<const float4 *>(u), a1 = *reinterpret_cast<const float4 *>(u + 4);
            const float4 b0 = *reinterpret_cast<const float4 *>(u + ug.W),
                         b1 = *reinterpret_cast<const float4 *>(u + ug.W + 4);
            gv = make_float4((a0.x + a0.y) + (b0.x + b0.y), (a0.z + a0.w) + (b0.z + b0.w),
                             (a1.x + a1.y) + (b1.x + b1.y), (a1.z + a1.w) + (b1.z + b1.w));
        } else {
            gv = *reinterpret_cast<const float4 *>(static_cast<const float *>(g.p) + n * g.bs + r);
            if (pg.p != nullptr) {
                const float2 q = *reinterpret_cast<const float2 *>(
                    static_cast<const float *>(pg.p) + n * pg.bs + (size_t)c * pg.H * pg.W +
                    (size_t)(yy / 2) * pg.W + xx / 2);
                gv.x += 0.25f * q.x;
                gv.y += 0.25f * q.x;
                gv.z += 0.25f * q.y;
                gv.w += 0.25f * q.y;
            }
        }
        float yv[4];
        if constexpr (sizeof(TA) == 2) {
            const uint2 yb = *reinterpret_cast<const uint2 *>(static_cast<const TA *>(y.p) + n * y.bs + r);
            yv[0] = __uint_as_float(yb.x << 16);
            yv[1] = __uint_as_float(yb.x & 0xffff0000u);
            yv[2] = __uint_as_float(yb.y << 16);
            yv[3] = __uint_as_float(yb.y & 0xffff0000u);
        } else {
            const float4 yf = *reinterpret_cast<const float4 *>(static_cast<const TA *>(y.p) + n * y.bs + r);
            yv[0] = yf.x; yv[1] = yf.y; yv[2] = yf.z; yv[3] = yf.w;
        }
        const float4 v = make_float4(yv[0] > 0.f ? gv.x : 0.f, yv[1] > 0.f ? gv.y : 0.f, yv[2] > 0.f ? gv.z : 0.f,
                                     yv[3] > 0.f ? gv.w : 0.f);
        sum = (v.x + v.y) + (v.z + v.w);
        if (dz) *reinterpret_cast<float4 *>(dz + i) = v;
        if (dzh) {
            const __bf16 h0 = (__bf16)v.x, h1 = (__bf16)v.y, h2 = (__bf16)v.z, h3 = (__bf16)v.w;
            uint2 o;
            o.x = (uint32_t)__builtin_bit_cast(unsigned short, h0) |
                  (uint32_t)__builtin_bit_cast(unsigned short, h1) << 16;
            o.y = (uint32_t)__builtin_bit_cast(unsigned short, h2) |
                  (uint32_t)__builtin_bit_cast(unsigned short, h3) << 16;
            *reinterpret_cast<uint2 *>(dzh + i) = o;
        }
    }
    const float t = wg_sum256(sum, sh4);
    if (threadIdx.x == 0) part[((size_t)c * N + n) * gridDim.x + blockIdx.x] = t;
}

// ------------------------------------------------------ pool / upsample
template <class TA>
__global__ void k_pool(View in, View out, int N, int C) {
    const uint32_t Ho = out.H, Wo = out.W;
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Ho * Wo) return;
    const uint32_t y = p / Wo, x = p - y * Wo, c = blockIdx.y, n = blockIdx.z;
    const TA *s = static_cast<const TA *>(in.p) + n * in.bs + (size_t)c * in.H * in.W;
    const float v = 0.25f * ((tof(s[(2 * y) * in.W + 2 * x]) + tof(s[(2 * y) * in.W + 2 * x + 1])) +
                             (tof(s[(2 * y + 1) * in.W + 2 * x]) + tof(s[(2 * y + 1) * in.W + 2 * x + 1])));
    static_cast<TA *>(out.p)[n * out.bs + (size_t)c * Ho * Wo + p] = fromf<TA>(v);
}

// gradient of pool: dx (fine, fp32) += dy (coarse) / 4
__global__ void k_pool_back_acc(View dy, View dx, int N, int C) {
    const uint32_t H = dx.H, W = dx.W;
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= H * W) return;
    const uint32_t y = p / W, x = p - y * W, c = blockIdx.y, n = blockIdx.z;
    const float g = static_cast<const float *>(dy.p)[n * dy.bs + (size_t)c * dy.H * dy.W + (size_t)(y / 2) * dy.W + x / 2];
    static_cast<float *>(dx.p)[n * dx.bs + (size_t)c * H * W + p] += 0.25f * g;
}

// The same, four fine pixels of a row per thread (W % 4 == 0, aligned planes).
__global__ void k_pool_back_acc4(View dy, View dx, int N, int C) {
    const uint32_t H = dx.H, W = dx.W;
    const uint32_t p = 4u * (blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= H * W) return;
    const uint32_t y = p / W, x = p - y * W, c = blockIdx.y, n = blockIdx.z;
    const float2 g = *reinterpret_cast<const float2 *>(static_cast<const float *>(dy.p) + n * dy.bs +
                                                       (size_t)c * dy.H * dy.W + (size_t)(y / 2) * dy.W + x / 2);
    float4 *d = reinterpret_cast<float4 *>(static_cast<float *>(dx.p) + n * dx.bs + (size_t)c * H * W + p);
    float4 v = *d;
    v.x += 0.25f * g.x;
    v.y += 0.25f * g.x;
    v.z += 0.25f * g.y;
    v.w += 0.25f * g.y;
    *d = v;
}

template <class TA>
__global__ void k_up(View in, View out, int N, int C) {
    const uint32_t H = out.H, W = out.W;
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= H * W) return;
    const uint32_t y = p / W, x = p - y * W, c = blockIdx.y, n = blockIdx.z;
    static_cast<TA *>(out.p)[n * out.bs + (size_t)c * H * W + p] =
        static_cast<const TA *>(in.p)[n * in.bs + (size_t)c * in.H * in.W + (size_t)(y / 2) * in.W + x / 2];
}

// The same, four fine pixels of a row per thread (W % 4 == 0, aligned planes):
// two coarse values in, each written twice.
template <class TA>
__global__ void k_up4(View in, View out, int N, int C) {
    const uint32_t H = out.H, W = out.W;
    const uint32_t p = 4u * (blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= H * W) return;
    const uint32_t y = p / W, x = p - y * W, c = blockIdx.y, n = blockIdx.z;
    const TA *src = static_cast<const TA *>(in.p) + n * in.bs + (size_t)c * in.H * in.W + (size_t)(y / 2) * in.W + x / 2;
    TA *dst = static_cast<TA *>(out.p) + n * out.bs + (size_t)c * H * W + p;
    if constexpr (sizeof(TA) == 2) {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(src);
        *reinterpret_cast<uint2 *>(dst) = make_uint2((v & 0xffffu) * 0x10001u, (v >> 16) * 0x10001u);
    } else {
        const float2 v = *reinterpret_cast<const float2 *>(src);
        *reinterpret_cast<float4 *>(dst) = make_float4(v.x, v.x, v.y, v.y);
    }
}

// gradient of upsample: dx (coarse, fp32) = sum of the 2x2 block of dy
__global__ void k_up_back(View dy, View dx, int N, int C) {
    const uint32_t Ho = dx.H, Wo = dx.W;
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= Ho * Wo) return;
    const uint32_t y = p / Wo, x = p - y * Wo, c = blockIdx.y, n = blockIdx.z;
    const float *s = static_cast<const float *>(dy.p) + n * dy.bs + (size_t)c * dy.H * dy.W;
    const float v = (s[(2 * y) * dy.W + 2 * x] + s[(2 * y) * dy.W + 2 * x + 1]) +
                    (s[(2 * y + 1) * dy.W + 2 * x] + s[(2 * y + 1) * dy.W + 2 * x + 1]);
    static_cast<float *>(dx.p)[n * dx.bs + (size_t)c * Ho * Wo + p] = v;
}

// ---------------------------------------------------------- 1x1 output
template <class TA>
__global__ void k_conv1x1(View in, const float *__restrict__ w, const float *__restrict__ b, int N, int cin,
                          int cout, float *__restrict__ out) {
    const size_t HW = (size_t)in.H * in.W;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)N * HW) return;
    const size_t n = i / HW, p = i % HW;
    const TA *s = static_cast<const TA *>(in.p) + n * in.bs + p;
    // four outputs per pass over the input planes (the layer has 3), the
    // sums in channel order as before
    for (int o0 = 0; o0 < cout; o0 += 4) {
        float acc[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[j] = o0 + j < cout ? b[o0 + j] : 0.f;
#pragma unroll 8
        for (int c = 0; c < cin; ++c) {
            const float xc = tof(s[(size_t)c * HW]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (o0 + j < cout) acc[j] += w[(o0 + j) * cin + c] * xc;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (o0 + j < cout) out[(n * cout + o0 + j) * HW + p] = acc[j];
    }
}

// gradient of 1x1 input: dx[c] = sum_o w[o][c] g[o]; layers with at most 4
// outputs keep their gradients in registers across the channels
__global__ void k_conv1x1_dx(const float *__restrict__ g, const float *__restrict__ w, int N, int cin, int cout,
                             int HW, View dx) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)N * HW) return;
    const size_t n = i / HW, p = i % HW;
    float *__restrict__ d = static_cast<float *>(dx.p) + n * dx.bs + p;
    if (cout <= 4) {
        float gv[4];
#pragma unroll
        for (int o = 0; o < 4; ++o) gv[o] = o < cout ? g[(n * cout + o) * HW + p] : 0.f;
#pragma unroll 4
        for (int c = 0; c < cin; ++c) {
            float acc = 0.f;
#pragma unroll
            for (int o = 0; o < 4; ++o)
                if (o < cout) acc += w[o * cin + c] * gv[o];
            d[(size_t)c * HW] = acc;
        }
        return;
    }
    for (int c = 0; c < cin; ++c) {
        float acc = 0.f;
        for (int o = 0; o < cout; ++o) acc += w[o * cin + c] * g[(n * cout + o) * HW + p];
        d[(size_t)c * HW] = acc;
    }
}

// 1x1 weight and bias gradients: one workgroup per (o, c) entry, and c = cin
// for the bias; fixed tree.
// dW[o][c] = sum of g[n][o](p) x[n][c](p), db[o] = sum of g[n][o](p) (pair c =
// cin), in two passes with a fixed order: workgroup (pair, b) sums its
// contiguous share of the N * HW products (fixed tree) into part[pair][b],
// then k_pair_final adds the BIAS_PARTS shares of each pair in order.
constexpr int BIAS_PARTS = 64;
template <class TA>
__global__ void __launch_bounds__(256) k_conv1x1_dw_partial(View x, const float *__restrict__ g, int N, int cin,
                                                            int cout, float *__restrict__ part) {
    __shared__ float sh[256];
    const int pair = blockIdx.x, b = blockIdx.y;
    const int o = pair / (cin + 1), c = pair % (cin + 1);
    const size_t HW = (size_t)x.H * x.W, total = (size_t)N * HW;
    const size_t len = (total + BIAS_PARTS - 1) / BIAS_PARTS;
    const size_t e0 = (size_t)b * len, e1 = min(total, e0 + len);
    const TA *__restrict__ xp = static_cast<const TA *>(x.p);
    float s = 0.f;
    size_t e = e0 + threadIdx.x;
    if (e < e1) {
        // (sample, pixel) of e, advanced by 256 each pass instead of divided
        uint32_t n = (uint32_t)(e / HW), p = (uint32_t)(e % HW);
        for (; e < e1; e += 256) {
            const float gv = g[((size_t)n * cout + o) * HW + p];
            s += c < cin ? gv * tof(xp[(size_t)n * x.bs + (size_t)c * HW + p]) : gv;
            p += 256;
            while (p >= (uint32_t)HW) { p -= (uint32_t)HW; ++n; }
        }
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) sh[threadIdx.x] += sh[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[(size_t)pair * BIAS_PARTS + b] = sh[0];
}

__global__ void k_conv1x1_dw_final(const float *__restrict__ part, int cin, int cout, float *__restrict__ dw,
                                   float *__restrict__ db) {
    const int pair = blockIdx.x * blockDim.x + threadIdx.x;
    if (pair >= cout * (cin + 1)) return;
    float s = 0.f;
    for (int b = 0; b < BIAS_PARTS; ++b) s += part[(size_t)pair * BIAS_PARTS + b];
    const int o = pair / (cin + 1), c = pair % (cin + 1);
    if (c < cin) dw[o * cin + c] = s;
    else db[o] = s;
}

// ------------------------------------------------------------ loss, Adam
// Count of fluid nodes times channels and the sum of squared errors, in FP64
// partials per workgroup (fixed order), then the gradient 2 (y - t) m / count.
__global__ void __launch_bounds__(256) k_loss_partial(const float *__restrict__ y, const float *__restrict__ t,
                                                      const uint8_t *__restrict__ mask, int N, int C, int HW,
                                                      double *__restrict__ part) {
    __shared__ double sh[2][256];
    double se = 0.0, cnt = 0.0;
    const size_t total = (size_t)N * HW;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (size_t)gridDim.x * 256) {
        if (!mask[i]) continue;
        const size_t n = i / HW, p = i % HW;
        for (int c = 0; c < C; ++c) {
            const double d = (double)y[(n * C + c) * HW + p] - (double)t[(n * C + c) * HW + p];
            se += d * d;
        }
        cnt += C;
    }
    sh[0][threadIdx.x] = se;
    sh[1][threadIdx.x] = cnt;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + k];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + k];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sh[0][0];
        part[2 * blockIdx.x + 1] = sh[1][0];
    }
}

__global__ void k_loss_final(const double *__restrict__ part, int n, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double se = 0.0, cnt = 0.0;
    for (int k = 0; k < n; ++k) {
        se += part[2 * k];
        cnt += part[2 * k + 1];
    }
    out[0] = cnt > 0 ? se / cnt : 0.0;
    out[1] = cnt;
}

__global__ void k_loss_grad(const float *__restrict__ y, const float *__restrict__ t, const uint8_t *__restrict__ mask,
                            int N, int C, int HW, const double *__restrict__ stats, float *__restrict__ g) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)N * C * HW) return;
    const size_t p = i % HW, n = i / ((size_t)C * HW);
    const float scale = (float)(2.0 / stats[1]);
    g[i] = mask[n * HW + p] ? scale * (y[i] - t[i]) : 0.f;
}

// Adam (Kingma & Ba 2015) with bias correction; c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void k_adam(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_zero(float *__restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// ------------------------------------------------------- conv 3x3 on MFMA
// bf16 activations and weights, FP32 accumulation: out[co][p] = bias[co] +
// sum over taps t and input channels ci of W[co][ci][t] x[ci][p + d_t], as a
// GEMM per tap with M = output channels, N = pixels, K = input channels, on
// v_mfma_f32_16x16x32_bf16.  Operand layout of that instruction (checked on
// the device): lane l holds A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16]
// for e = 0..7 and receives D[4 (l / 16) + r][l % 16] for r = 0..3.
//
// A workgroup (4 waves) computes an 8 x 32 pixel tile for 64 output channels;
// wave w owns pixel rows 2w and 2w + 1 (four 16-pixel N tiles) and all four
// 16-channel M tiles.  Input channels are staged 32 at a time through LDS
// channel-last ([y][x][ci], 40 bf16 per pixel so that the 16-byte fragment
// reads of 16 consecutive pixels fall in distinct banks), with the one-pixel
// halo (periodic x, zero y); the packed weights ([t][co][ci], see
// k_pack_all) likewise.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int MH = 8, MCI = 32, MPS = 40;

// Packed bf16 weights of every 3x3 matrix-core layer in one launch (workgroup
// row y packs job y).  Forward layout Wp[t][co][ci] from W[co][ci][t], ci
// padded with zeros to pad; flipped layout W'[t][ci][co] = W[co][ci][8 - t],
// co padded: the weights of the input-gradient convolution.
__global__ void __launch_bounds__(256) k_pack_all(const float *__restrict__ theta, __bf16 *__restrict__ base,
                                                  PackJobs jobs) {
    const PackJob j = jobs.job[blockIdx.y];
    const int n = 9 * j.rows * j.pad;   // rows: cout (forward) or cin (flipped)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int k = i % j.pad, r = (i / j.pad) % j.rows, t = i / (j.pad * j.rows);
        const float *w = theta + j.woff;
        float v;
        if (j.flip) v = k < j.cout ? w[((size_t)k * j.cin + r) * 9 + (8 - t)] : 0.f;   // k = co, r = ci
        else v = k < j.cin ? w[((size_t)r * j.cin + k) * 9 + t] : 0.f;                  // k = ci, r = co
        base[j.out + i] = (__bf16)v;
    }
}

// Tile of k_conv3x3_mfma: MH rows x TWD columns of one sample, computed by
// TWD / 4 waves (NT threads); each wave owns four 16-pixel N tiles (two rows
// of 32 columns, or one row of 64).
template <int TWD>
struct ConvTile {
    static_assert(TWD == 32 || TWD == 64, "tile width 32 or 64");
    static constexpr int TW = TWD, NT = 8 * TWD, QR = TWD / 16, RPW = 4 / QR;
};

// Staging of one 32-channel chunk of the input tile (rows ty0 - 1 .. ty0 + MH,
// columns tx0 - 1 .. tx0 + TW, periodic in x, zero outside the rows and
// channels) and of its packed weights, in two halves: load() issues the
// global loads into registers, store() writes them to LDS (channel-last,
// MPS bf16 per pixel).  The loads of chunk k + 1 are issued before the
// products of chunk k, so they are in flight while the matrix cores work.
//
// VEC (rows of whole 8-pixel groups: W % 8 == 0, 16-byte aligned planes): a
// task is 8 channels x 8 pixels of one row, eight 16-byte loads (one per
// channel plane) transposed in registers into eight 16-byte LDS stores (one
// per pixel); the halo columns tx0 - 1 and tx0 + TW are tasks of 8 channels
// x 1 pixel; at most one task per thread.  Otherwise each thread gathers 8
// channels of a pixel with 2-byte loads, XT pixels per thread.
template <int NM, bool VEC, int TWD>
struct ConvStage {
    using T = ConvTile<TWD>;
    static constexpr int TW = T::TW, NT = T::NT, CO = 16 * NM;
    static constexpr int XTASKS = (MCI / 8) * (MH + 2) * (TW + 2), XT = (XTASKS + NT - 1) / NT;
    static constexpr int WTASKS = 9 * CO * (MCI / 8), WT = (WTASKS + NT - 1) / NT;
    static constexpr int VIN = (MCI / 8) * (MH + 2) * (TW / 8);   // 8 x 8 tasks
    static constexpr int VHALO = (MCI / 8) * (MH + 2) * 2;        // 8 x 1 tasks
    static_assert(!VEC || VIN + VHALO <= NT, "one vector staging task per thread");
    uint4 v[VEC ? 8 : 1];              // VEC: 8 channel planes x 8 pixels
    uint32_t hv[VEC ? 8 : 1];          // VEC: 8 channels of a halo pixel
    bf16x8 xv[VEC ? 1 : XT];
    uint4 wv[WT];
    uint32_t vmask = 0u, xmask[VEC ? 1 : XT] = {}, wmask = 0u;   // loaded values that are real

    __device__ __forceinline__ static int wrap(int x, int W) {
        if (x < 0) x += W;
        if (x >= W) x -= W;
        if (x >= W) x %= W;                  // lattices narrower than a tile
        return x;
    }

    __device__ __forceinline__ void load(const __bf16 *__restrict__ xin, const __bf16 *__restrict__ wp, int H,
                                         int W, int tx0, int ty0, int ci0, int cin, int cout, int co0, int cin_pad,
                                         int tid) {
        // 32-bit offsets within the sample (its planes hold fewer than 2^31
        // values, checked when the network is made).  Every load is issued
        // (a value that is not needed comes from a clamped row and channel
        // and is replaced by zero in store(), when it has arrived): loads
        // under a condition, or values cleared right after their load, make
        // the compiler split the loads up or wait for each one; clamping
        // rather than one fixed address keeps those loads from all landing
        // on one cache line.
        const uint32_t HW = (uint32_t)(H * W);
        if constexpr (VEC) {
            if (tid < VIN) {
                const int g = tid % (TW / 8), r = (tid / (TW / 8)) % (MH + 2), c8 = tid / ((TW / 8) * (MH + 2));
                const int y = ty0 - 1 + r;
                const int x = wrap(tx0 + 8 * g, W);
                const bool oky = y >= 0 && y < H;
                const uint32_t pix = (uint32_t)(min(max(y, 0), H - 1) * W + x);
                vmask = 0u;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = ci0 + 8 * c8 + j;
                    const bool ok = oky && c < cin;
                    v[j] = *reinterpret_cast<const uint4 *>(xin + (uint32_t)min(c, cin - 1) * HW + pix);
                    vmask |= (ok ? 1u : 0u) << j;
                }
            } else if (tid < VIN + VHALO) {
                const int h = tid - VIN;
                const int side = h % 2, r = (h / 2) % (MH + 2), c8 = h / (2 * (MH + 2));
                const int y = ty0 - 1 + r;
                const int x = wrap(side ? tx0 + TW : tx0 - 1, W);
                const bool oky = y >= 0 && y < H;
                const uint32_t pix = (uint32_t)(min(max(y, 0), H - 1) * W + x);
                const unsigned short *__restrict__ xs16 = reinterpret_cast<const unsigned short *>(xin);
                vmask = 0u;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = ci0 + 8 * c8 + j;
                    const bool ok = oky && c < cin;
                    hv[j] = xs16[(uint32_t)min(c, cin - 1) * HW + pix];
                    vmask |= (ok ? 1u : 0u) << j;
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < XT; ++k) {
                const int e = tid + NT * k;
                const int q = e % (TW + 2), r = (e / (TW + 2)) % (MH + 2), c8 = e / ((TW + 2) * (MH + 2));
                const int y = ty0 - 1 + r;
                const int x = wrap(tx0 - 1 + q, W);
                const bool oky = e < XTASKS && y >= 0 && y < H;
                const uint32_t pix = (uint32_t)(min(max(y, 0), H - 1) * W + x);
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = ci0 + 8 * c8 + j;
                    const bool ok = oky && c < cin;
                    xv[k][j] = xin[(uint32_t)min(c, cin - 1) * HW + pix];
                    xmask[k] = (xmask[k] & ~(1u << j)) | (ok ? 1u : 0u) << j;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < WT; ++k) {
            const int e = tid + NT * k;
            const int c8 = e % (MCI / 8), co = (e / (MCI / 8)) % CO, t = e / ((MCI / 8) * CO);
            const bool ok = e < WTASKS && co0 + co < cout;
            wv[k] = *reinterpret_cast<const uint4 *>(wp + ((size_t)min(t, 8) * cout + min(co0 + co, cout - 1)) * cin_pad + ci0 + 8 * c8);
            wmask = (wmask & ~(1u << k)) | (ok ? 1u : 0u) << k;
        }
    }

    __device__ __forceinline__ void store(__bf16 *xs, __bf16 *ws, int tid) const {
        if constexpr (VEC) {
            if (tid < VIN) {
                const int g = tid % (TW / 8), r = (tid / (TW / 8)) % (MH + 2), c8 = tid / ((TW / 8) * (MH + 2));
                uint4 w[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) w[j] = (vmask >> j & 1u) ? v[j] : make_uint4(0u, 0u, 0u, 0u);
                // w[j] holds pixels 2d, 2d + 1 of channel j in dword d; pixel p's
                // eight channels go out as one 16-byte word (channel 2m in the
                // low half of dword m)
                const uint32_t *u = reinterpret_cast<const uint32_t *>(w);
#pragma unroll
                for (int p = 0; p < 8; ++p) {
                    const uint32_t sel = (p & 1) ? 0x07060302u : 0x05040100u;
                    const int d = p >> 1;
                    uint4 o;
                    o.x = __builtin_amdgcn_perm(u[4 * 1 + d], u[4 * 0 + d], sel);
                    o.y = __builtin_amdgcn_perm(u[4 * 3 + d], u[4 * 2 + d], sel);
                    o.z = __builtin_amdgcn_perm(u[4 * 5 + d], u[4 * 4 + d], sel);
                    o.w = __builtin_amdgcn_perm(u[4 * 7 + d], u[4 * 6 + d], sel);
                    *reinterpret_cast<uint4 *>(&xs[(r * (TW + 2) + 1 + 8 * g + p) * MPS + 8 * c8]) = o;
                }
            } else if (tid < VIN + VHALO) {
                const int h = tid - VIN;
                const int side = h % 2, r = (h / 2) % (MH + 2), c8 = h / (2 * (MH + 2));
                const int q = side ? TW + 1 : 0;
                uint32_t hz[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) hz[j] = (vmask >> j & 1u) ? hv[j] & 0xffffu : 0u;
                *reinterpret_cast<uint4 *>(&xs[(r * (TW + 2) + q) * MPS + 8 * c8]) =
                    make_uint4(hz[0] | hz[1] << 16, hz[2] | hz[3] << 16, hz[4] | hz[5] << 16, hz[6] | hz[7] << 16);
            }
        } else {
#pragma unroll
            for (int k = 0; k < XT; ++k) {
                const int e = tid + NT * k;
                if (e < XTASKS) {
                    const int q = e % (TW + 2), r = (e / (TW + 2)) % (MH + 2), c8 = e / ((TW + 2) * (MH + 2));
                    bf16x8 o = xv[k];
#pragma unroll
                    for (int j = 0; j < 8; ++j)
                        if (!(xmask[k] >> j & 1u)) o[j] = (__bf16)0.f;
                    *reinterpret_cast<bf16x8 *>(&xs[(r * (TW + 2) + q) * MPS + 8 * c8]) = o;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < WT; ++k) {
            const int e = tid + NT * k;
            if (e < WTASKS) {
                const int c8 = e % (MCI / 8), co = (e / (MCI / 8)) % CO, t = e / ((MCI / 8) * CO);
                *reinterpret_cast<uint4 *>(&ws[(t * CO + co) * MPS + 8 * c8]) =
                    (wmask >> k & 1u) ? wv[k] : make_uint4(0u, 0u, 0u, 0u);
            }
        }
    }
};

// LDS of the convolution: the staged input tile and weights, reused after the
// channel loop for the output tile (CO rows of OS values) on its way to
// 16-byte stores.
template <class TO, int NM, int TWD>
struct ConvLds {
    static constexpr int CO = 16 * NM, TW = TWD;
    static constexpr int XS = (MH + 2) * (TW + 2) * MPS, WS = 9 * CO * MPS;   // bf16
    static constexpr int OS = MH * TW + 16 / (int)sizeof(TO);                 // output row stride
    static constexpr int IN_BYTES = 2 * (XS + WS), OUT_BYTES = CO * OS * (int)sizeof(TO);
    static constexpr int BYTES = IN_BYTES > OUT_BYTES ? IN_BYTES : OUT_BYTES;
};

// Input: bf16 activations (or the bf16 copy of the layer gradient); TO:
// output type; bias may be NULL.  NM: 16-channel output tiles per workgroup
// (4: 64 channels; 2: 32 channels).  VEC: see ConvStage; it also sends the
// output tile through LDS so that each lane stores 16 contiguous bytes of one
// plane.  TWD: tile width (32, or 64 with 512 threads, which halves the
// staged weight bytes per output).
//
// pool.p != NULL (bf16 output, VEC, even H and W): the epilogue also writes
// the 2 x 2 means of the output tile to pool (H / 2 x W / 2 planes), with the
// arithmetic of k_pool on the same bf16 values, so the separate pooling pass
// is not needed.  up.p != NULL (same conditions): the epilogue also writes the
// nearest 2x upsampling of the output tile to up (2H x 2W planes: each value
// copied to a 2 x 2 block), so the separate upsampling pass is not needed.
//
// Workgroups are dispatched round-robin over the 8 XCDs; block b is given
// tile b' = (b mod 8) * (nb / 8) + b / 8 so that each XCD computes a
// contiguous run of tiles, and the halo rows and the cache lines that
// neighbouring tiles share, and the weights, stay in its L2.
template <class TO, int NM, bool VEC, int TWD>
__global__ void __launch_bounds__(ConvTile<TWD>::NT) k_conv3x3_mfma(View in, const __bf16 *__restrict__ wp,
                                                                     const float *__restrict__ bias, View out,
                                                                     View pool, View up, int cin, int cout,
                                                                     int cin_pad, int relu) {
    using L = ConvLds<TO, NM, TWD>;
    using T = ConvTile<TWD>;
    constexpr int CO = L::CO, TW = T::TW, NT = T::NT;
    __shared__ __attribute__((aligned(16))) char lds[L::BYTES];
    __bf16 *xs = reinterpret_cast<__bf16 *>(lds);
    __bf16 *ws = xs + L::XS;
    const int H = in.H, W = in.W;
    int bxy;
    {
        const int nb = gridDim.x * gridDim.y, b = blockIdx.x + gridDim.x * blockIdx.y;
        const int full = nb / 8 * 8;
        bxy = b < full ? (b % 8) * (full / 8) + b / 8 : b;
    }
    const int bx = bxy % gridDim.x, by = bxy / gridDim.x;
    const int tiles_x = (W + TW - 1) / TW;
    const int tx0 = (bx % tiles_x) * TW, ty0 = (bx / tiles_x) * MH;
    const int ncob = (cout + CO - 1) / CO;
    const int n = by / ncob, co0 = (by % ncob) * CO;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    const __bf16 *__restrict__ xin = static_cast<const __bf16 *>(in.p) + (size_t)n * in.bs;
    // The lane's biases, read before the channel loop: loaded in the epilogue
    // they would put a wait for memory (which on this architecture also waits
    // for every store before it) in front of each of the output stores.
    float bv[NM][4];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + 16 * m + (lane >> 4) * 4 + r;
            bv[m][r] = (bias != nullptr && co < cout) ? bias[co] : 0.f;
        }
    f32x4 acc[NM][4];
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[m][q] = f32x4{0.f, 0.f, 0.f, 0.f};
    ConvStage<NM, VEC, TWD> st;
    st.load(xin, wp, H, W, tx0, ty0, 0, cin, cout, co0, cin_pad, tid);
    // (cin >= 1: a loop that always runs once lets its wait for the staged
    // loads cover the bias loads too, so the epilogue's stores need no waits.)
    int ci0 = 0;
    do {
        st.store(xs, ws, tid);
        __syncthreads();
        if (ci0 + MCI < cin) st.load(xin, wp, H, W, tx0, ty0, ci0 + MCI, cin, cout, co0, cin_pad, tid);
#pragma unroll 1
        for (int t = 0; t < 9; ++t) {
            const int dy = t / 3, dx = t % 3;
            bf16x8 a[NM];
#pragma unroll
            for (int m = 0; m < NM; ++m)
                a[m] = *reinterpret_cast<const bf16x8 *>(&ws[(t * CO + 16 * m + lr) * MPS + lk]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int pr = T::RPW * wave + q / T::QR, pc = (q % T::QR) * 16 + lr;
                const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&xs[((pr + dy) * (TW + 2) + pc + dx) * MPS + lk]);
#pragma unroll
                for (int m = 0; m < NM; ++m) acc[m][q] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], b, acc[m][q], 0, 0, 0);
            }
        }
        __syncthreads();
        ci0 += MCI;
    } while (ci0 < cin);
    TO *__restrict__ yo = static_cast<TO *>(out.p) + (size_t)n * out.bs;
    if constexpr (VEC) {
        // D[4 (l / 16) + r][l % 16] of tile (m, q) -> LDS row co, then each
        // lane stores 16 bytes of one output row of one plane
        TO *os = reinterpret_cast<TO *>(lds);
#pragma unroll
        for (int m = 0; m < NM; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int col = 16 * m + (lane >> 4) * 4 + r;
                    const int pix = (T::RPW * wave + q / T::QR) * TW + (q % T::QR) * 16 + lr;
                    float v = acc[m][q][r] + bv[m][r];
                    if (relu) v = fmaxf(v, 0.f);
                    os[col * L::OS + pix] = fromf<TO>(v);
                }
        __syncthreads();
        constexpr int EPP = 16 / (int)sizeof(TO), PPR = TW / EPP, PIECES = CO * MH * PPR;
        const uint32_t HW = (uint32_t)(H * W);
#pragma unroll
        for (int k = 0; k < (PIECES + NT - 1) / NT; ++k) {
            const int e = tid + NT * k;
            const int kk = e % PPR, row = (e / PPR) % MH, col = e / (PPR * MH);
            const int y = ty0 + row, x = tx0 + kk * EPP, co = co0 + col;
            if (e < PIECES && co < cout && y < H && x < W) {
                const uint4 v = *reinterpret_cast<const uint4 *>(&os[col * L::OS + row * TW + kk * EPP]);
                *reinterpret_cast<uint4 *>(yo + (uint32_t)co * HW + (uint32_t)(y * W + x)) = v;
                if constexpr (sizeof(TO) == 2) {
                    if (up.p != nullptr) {
                        // eight values -> sixteen (each twice) in rows 2 y and 2 y + 1
                        auto dup = [](uint32_t w) {
                            return make_uint2((w & 0xffffu) * 0x10001u, (w >> 16) * 0x10001u);
                        };
                        const uint2 d0 = dup(v.x), d1 = dup(v.y), d2 = dup(v.z), d3 = dup(v.w);
                        const uint4 lo = make_uint4(d0.x, d0.y, d1.x, d1.y), hi = make_uint4(d2.x, d2.y, d3.x, d3.y);
                        TO *uo = static_cast<TO *>(up.p) + (size_t)n * up.bs +
                                 (size_t)co * ((uint32_t)up.H * (uint32_t)up.W) + (uint32_t)(2 * y * up.W + 2 * x);
                        *reinterpret_cast<uint4 *>(uo) = lo;
                        *reinterpret_cast<uint4 *>(uo + 8) = hi;
                        *reinterpret_cast<uint4 *>(uo + up.W) = lo;
                        *reinterpret_cast<uint4 *>(uo + up.W + 8) = hi;
                    }
                }
            }
        }
        if constexpr (sizeof(TO) == 2) {
            if (pool.p != nullptr) {
                // eight pooled values (16 bytes) of one pooled row per piece,
                // from two 16-value runs of output rows 2 r and 2 r + 1
                constexpr int PPR2 = TW / 16, PP = CO * (MH / 2) * PPR2;
                const uint32_t HWo = (uint32_t)(pool.H * pool.W);
                TO *__restrict__ po = static_cast<TO *>(pool.p) + (size_t)n * pool.bs;
#pragma unroll
                for (int k = 0; k < (PP + NT - 1) / NT; ++k) {
                    const int e = tid + NT * k;
                    const int kk = e % PPR2, r = (e / PPR2) % (MH / 2), col = e / (PPR2 * (MH / 2));
                    const int y = ty0 / 2 + r, x = tx0 / 2 + 8 * kk, co = co0 + col;
                    if (e < PP && co < cout && y < pool.H && x < pool.W) {
                        const TO *r0 = &os[col * L::OS + (2 * r) * TW + 16 * kk], *r1 = r0 + TW;
                        uint32_t w4[4];
#pragma unroll
                        for (int j = 0; j < 4; ++j) {
                            const float a0 = 0.25f * ((tof(r0[4 * j]) + tof(r0[4 * j + 1])) +
                                                      (tof(r1[4 * j]) + tof(r1[4 * j + 1])));
                            const float a1 = 0.25f * ((tof(r0[4 * j + 2]) + tof(r0[4 * j + 3])) +
                                                      (tof(r1[4 * j + 2]) + tof(r1[4 * j + 3])));
                            w4[j] = (uint32_t)__builtin_bit_cast(unsigned short, fromf<TO>(a0)) |
                                    (uint32_t)__builtin_bit_cast(unsigned short, fromf<TO>(a1)) << 16;
                        }
                        *reinterpret_cast<uint4 *>(po + (uint32_t)co * HWo + (uint32_t)(y * pool.W + x)) =
                            make_uint4(w4[0], w4[1], w4[2], w4[3]);
                    }
                }
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < NM; ++m)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int y = ty0 + T::RPW * wave + q / T::QR, x = tx0 + (q % T::QR) * 16 + lr;
                if (y >= H || x >= W) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = co0 + 16 * m + (lane >> 4) * 4 + r;
                    if (co >= cout) continue;
                    float v = acc[m][q][r] + bv[m][r];
                    if (relu) v = fmaxf(v, 0.f);
                    yo[(size_t)co * H * W + (size_t)y * W + x] = fromf<TO>(v);
                }
            }
    }
}

// Weight gradient on matrix cores (bf16 build, 3x3 layers after the first):
// for each tap (dy, dx), dW[co][ci] = sum over pixels p of dz[co](p)
// x[ci](p + (dy - 1, dx - 1)), a product with K = pixels, where dz is the layer
// gradient rounded to bf16 by k_relu_mask.  A workgroup owns 32
// output x 32 input channels (a 2 x 2 grid of waves, 16 x 16 each, all nine
// taps in 36 accumulation registers) and walks a chunk of 4 x 32 pixel tiles.
// The lane's eight K values are eight consecutive pixels of one row, so the
// operands of the three column shifts come from one 16-byte LDS read of the
// staged input row plus one neighbouring dword each; each staged row r then
// serves the dz rows r - dy of the three row shifts.  Partials
// [chunk][co][ci][tap] are summed in a fixed order by k_sum_grads.
constexpr int DM_CO = 32, DM_CI = 32, DM_TR = 4, DM_TW = 32, DM_PX = DM_TR * DM_TW;
constexpr int DM_DZS = DM_PX + 8;                 // dz channel stride (bf16)
constexpr int DM_XR = DM_TW + 16;                 // staged x row: 8 | 32 pixels | 8, halo at 7 and 40
constexpr int DM_XSC = (DM_TR + 2) * DM_XR + 8;   // x channel stride (bf16)
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

// x column tx0 + c (c in [-1, 32]) as the staged tile holds it: periodic at
// both ends of the row; columns more than one past the last one feed no
// output pixel and hold zero (-1 returned).
__device__ __forceinline__ int dw_col(int tx0, int c, int W) {
    const int col = tx0 + c;
    if (col < 0) return W - 1;
    if (col == W) return 0;
    return col < W ? col : -1;
}

// Staging of one tile: each thread's share of the dz rows, the x rows and the
// x halo columns, loaded into registers in one batch (one wait for memory per
// tile) and written to LDS afterwards.  VEC: whole, aligned 32-pixel rows move
// as 16-byte loads; otherwise one value per load.
template <bool VEC>
struct DwStage {
    static constexpr int DZ_T = VEC ? (DM_CO * DM_TR * (DM_TW / 8) + 255) / 256 : (DM_CO * DM_PX + 255) / 256;
    static constexpr int X_T = VEC ? (DM_CI * (DM_TR + 2) * (DM_TW / 8) + 255) / 256
                                   : (DM_CI * (DM_TR + 2) * DM_TW + 255) / 256;
    static constexpr int H_T = (DM_CI * (DM_TR + 2) * 2 + 255) / 256;
    using V = typename std::conditional<VEC, bf16x8, __bf16>::type;
    V dzv[DZ_T], xv[X_T];
    __bf16 hv[H_T];
};

template <bool VEC>
__device__ __forceinline__ void dw_load(DwStage<VEC> &st, const View &x, const __bf16 *__restrict__ dz, int cin,
                                        int cout, int co0, int ci0, int tile, int tiles_x, int tiles_y, int tid) {
    const int H = x.H, W = x.W;
    const int n = tile / (tiles_x * tiles_y), rem = tile % (tiles_x * tiles_y);
    const int ty0 = (rem / tiles_x) * DM_TR, tx0 = (rem % tiles_x) * DM_TW;
    const __bf16 *__restrict__ xin = static_cast<const __bf16 *>(x.p) + (size_t)n * x.bs;
    const __bf16 *__restrict__ dzn = dz + (size_t)n * cout * H * W;
    const __bf16 zero = (__bf16)0.f;
    if constexpr (VEC) {
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::DZ_T; ++k) {
            const int e = tid + 256 * k;
            const int q = (e % (DM_TW / 8)) * 8, j = (e / (DM_TW / 8)) % DM_TR, o = e / (DM_TR * DM_TW / 8);
            const int y = ty0 + j;
            st.dzv[k] = bf16x8{zero, zero, zero, zero, zero, zero, zero, zero};
            if (e < DM_CO * DM_TR * (DM_TW / 8) && co0 + o < cout && y < H)
                st.dzv[k] = *reinterpret_cast<const bf16x8 *>(&dzn[(size_t)(co0 + o) * H * W + (size_t)y * W + tx0 + q]);
        }
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::X_T; ++k) {
            const int e = tid + 256 * k;
            const int q = (e % (DM_TW / 8)) * 8, r = (e / (DM_TW / 8)) % (DM_TR + 2), c = e / ((DM_TR + 2) * DM_TW / 8);
            const int y = ty0 - 1 + r;
            st.xv[k] = bf16x8{zero, zero, zero, zero, zero, zero, zero, zero};
            if (e < DM_CI * (DM_TR + 2) * (DM_TW / 8) && ci0 + c < cin && y >= 0 && y < H)
                st.xv[k] = *reinterpret_cast<const bf16x8 *>(&xin[(size_t)(ci0 + c) * H * W + (size_t)y * W + tx0 + q]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::DZ_T; ++k) {
            const int e = tid + 256 * k;
            const int o = e / DM_PX, p = e % DM_PX;
            const int y = ty0 + p / DM_TW, xx = tx0 + p % DM_TW;
            st.dzv[k] = zero;
            if (e < DM_CO * DM_PX && co0 + o < cout && y < H && xx < W)
                st.dzv[k] = dzn[(size_t)(co0 + o) * H * W + (size_t)y * W + xx];
        }
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::X_T; ++k) {
            const int e = tid + 256 * k;
            const int q = e % DM_TW, r = (e / DM_TW) % (DM_TR + 2), c = e / ((DM_TR + 2) * DM_TW);
            const int y = ty0 - 1 + r, col = dw_col(tx0, q, W);
            st.xv[k] = zero;
            if (e < DM_CI * (DM_TR + 2) * DM_TW && ci0 + c < cin && y >= 0 && y < H && col >= 0)
                st.xv[k] = xin[(size_t)(ci0 + c) * H * W + (size_t)y * W + col];
        }
    }
    // halo columns -1 and 32 of every staged row
#pragma unroll
    for (int k = 0; k < DwStage<VEC>::H_T; ++k) {
        const int e = tid + 256 * k;
        const int side = e & 1, r = (e >> 1) % (DM_TR + 2), c = (e >> 1) / (DM_TR + 2);
        const int y = ty0 - 1 + r, col = dw_col(tx0, side ? DM_TW : -1, W);
        st.hv[k] = zero;
        if (e < DM_CI * (DM_TR + 2) * 2 && ci0 + c < cin && y >= 0 && y < H && col >= 0)
            st.hv[k] = xin[(size_t)(ci0 + c) * H * W + (size_t)y * W + col];
    }
}

template <bool VEC>
__device__ __forceinline__ void dw_store(const DwStage<VEC> &st, __bf16 *dzs, __bf16 *xs, int tid) {
    if constexpr (VEC) {
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::DZ_T; ++k) {
            const int e = tid + 256 * k;
            if (e >= DM_CO * DM_TR * (DM_TW / 8)) continue;
            const int q = (e % (DM_TW / 8)) * 8, j = (e / (DM_TW / 8)) % DM_TR, o = e / (DM_TR * DM_TW / 8);
            *reinterpret_cast<bf16x8 *>(&dzs[o * DM_DZS + j * DM_TW + q]) = st.dzv[k];
        }
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::X_T; ++k) {
            const int e = tid + 256 * k;
            if (e >= DM_CI * (DM_TR + 2) * (DM_TW / 8)) continue;
            const int q = (e % (DM_TW / 8)) * 8, r = (e / (DM_TW / 8)) % (DM_TR + 2), c = e / ((DM_TR + 2) * DM_TW / 8);
            *reinterpret_cast<bf16x8 *>(&xs[c * DM_XSC + r * DM_XR + 8 + q]) = st.xv[k];
        }
    } else {
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::DZ_T; ++k) {
            const int e = tid + 256 * k;
            if (e >= DM_CO * DM_PX) continue;
            dzs[(e / DM_PX) * DM_DZS + e % DM_PX] = st.dzv[k];
        }
#pragma unroll
        for (int k = 0; k < DwStage<VEC>::X_T; ++k) {
            const int e = tid + 256 * k;
            if (e >= DM_CI * (DM_TR + 2) * DM_TW) continue;
            const int q = e % DM_TW, r = (e / DM_TW) % (DM_TR + 2), c = e / ((DM_TR + 2) * DM_TW);
            xs[c * DM_XSC + r * DM_XR + 8 + q] = st.xv[k];
        }
    }
#pragma unroll
    for (int k = 0; k < DwStage<VEC>::H_T; ++k) {
        const int e = tid + 256 * k;
        if (e >= DM_CI * (DM_TR + 2) * 2) continue;
        const int side = e & 1, r = (e >> 1) % (DM_TR + 2), c = (e >> 1) / (DM_TR + 2);
        xs[c * DM_XSC + r * DM_XR + (side ? 8 + DM_TW : 7)] = st.hv[k];
    }
}

// The tiles of a chunk are software-pipelined: the next tile's loads are in
// flight (in registers) while the current tile's products run from LDS.
template <bool VEC>
__global__ void __launch_bounds__(256) k_conv3x3_dw_mfma(View x, const __bf16 *__restrict__ dz, int N, int cin,
                                                         int cout, int tiles_per_chunk,
                                                         float *__restrict__ partial) {
    __shared__ __attribute__((aligned(16))) __bf16 dzs[DM_CO * DM_DZS];
    __shared__ __attribute__((aligned(16))) __bf16 xs[DM_CI * DM_XSC];
    const int H = x.H, W = x.W;
    const int tiles_x = (W + DM_TW - 1) / DM_TW, tiles_y = (H + DM_TR - 1) / DM_TR;
    const int ntiles = N * tiles_x * tiles_y;
    const int chunk = blockIdx.x, co0 = blockIdx.y * DM_CO, ci0 = blockIdx.z * DM_CI;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wco = (wave & 1) * 16, wci = (wave >> 1) * 16;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    f32x4 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int t_begin = chunk * tiles_per_chunk, t_end = min(ntiles, t_begin + tiles_per_chunk);
    DwStage<VEC> st;
    if (t_begin < t_end) dw_load<VEC>(st, x, dz, cin, cout, co0, ci0, t_begin, tiles_x, tiles_y, tid);
    for (int tile = t_begin; tile < t_end; ++tile) {
        dw_store<VEC>(st, dzs, xs, tid);
        __syncthreads();
        if (tile + 1 < t_end) dw_load<VEC>(st, x, dz, cin, cout, co0, ci0, tile + 1, tiles_x, tiles_y, tid);
        bf16x8 a[DM_TR];
#pragma unroll
        for (int j = 0; j < DM_TR; ++j)
            a[j] = *reinterpret_cast<const bf16x8 *>(&dzs[(wco + lr) * DM_DZS + j * DM_TW + lk]);
#pragma unroll
        for (int r = 0; r < DM_TR + 2; ++r) {
            const __bf16 *row = &xs[(wci + lr) * DM_XSC + r * DM_XR + 8 + lk];
            const u32x4 c = __builtin_bit_cast(u32x4, *reinterpret_cast<const bf16x8 *>(row));
            const uint32_t lw = *reinterpret_cast<const uint32_t *>(row - 2);   // pixels lk - 2, lk - 1
            const uint32_t rw = *reinterpret_cast<const uint32_t *>(row + 8);   // pixels lk + 8, lk + 9
            const uint32_t m1 = (c.x >> 16) | (c.y << 16), m2 = (c.y >> 16) | (c.z << 16),
                           m3 = (c.z >> 16) | (c.w << 16);
            const bf16x8 b[3] = {__builtin_bit_cast(bf16x8, u32x4{(lw >> 16) | (c.x << 16), m1, m2, m3}),
                                 __builtin_bit_cast(bf16x8, c),
                                 __builtin_bit_cast(bf16x8, u32x4{m1, m2, m3, (c.w >> 16) | (rw << 16)})};
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const int j = r - dy;
                if (j < 0 || j >= DM_TR) continue;
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    acc[dy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j], b[dx], acc[dy * 3 + dx], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 9; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = co0 + wco + (lane >> 4) * 4 + r, ci = ci0 + wci + lr;
            if (co < cout && ci < cin) partial[(((size_t)chunk * cout + co) * cin + ci) * 9 + t] = acc[t][r];
        }
}

inline unsigned nblk(size_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }
// (pixel blocks of 256, channel, sample) grid of the elementwise kernels
inline dim3 pix_grid(int H, int W, int C, int N) { return dim3(nblk((size_t)H * W), (unsigned)C, (unsigned)N); }

}  // namespace

// ------------------------------------------------------------ launchers
template <class TI, class TO>
hipError_t conv3x3(const View &in, const float *w, const float *bias, const View &out, int N, int cin, int cout,
                   bool relu, hipStream_t s) {
    const int tiles = ((in.W + TW - 1) / TW) * ((in.H + TH - 1) / TH);
    const dim3 grid(tiles, N * ((cout + CO_T - 1) / CO_T));
    k_conv3x3<TI, TO><<<grid, 256, 0, s>>>(in, w, bias, out, cin, cout, relu ? 1 : 0);
    return hipGetLastError();
}
template hipError_t conv3x3<float, float>(const View &, const float *, const float *, const View &, int, int, int, bool, hipStream_t);
template hipError_t conv3x3<float, __bf16>(const View &, const float *, const float *, const View &, int, int, int, bool, hipStream_t);
template hipError_t conv3x3<__bf16, __bf16>(const View &, const float *, const float *, const View &, int, int, int, bool, hipStream_t);

int pad32(int c) { return (c + MCI - 1) / MCI * MCI; }

// 32-channel output tiles for 32 or fewer output channels (a 64-channel tile
// would spend half its products on padding).
bool mfma_narrow(int cout) { return cout <= 32; }

// Whole 8-pixel groups and 16-byte aligned planes in and out: the vector
// staging and the 16-byte output stores of k_conv3x3_mfma.
template <class TO>
bool mfma_vec_ok(const View &in, const View &out) {
    const int epp = 16 / (int)sizeof(TO);
    return in.W % 8 == 0 && (uintptr_t)in.p % 16 == 0 && in.bs % 8 == 0 && (uintptr_t)out.p % 16 == 0 &&
           out.bs % epp == 0;
}

// Shape of a convolution launch: 64-column tiles (512 threads) where the
// rows are whole 64-column tiles and that still gives at least 256
// workgroups, else 32; 32-channel output tiles for at most 32 output
// channels or where 64-channel tiles would leave more than half of the 256
// CUs idle.
template <class TO, int NM, int TWD>
hipError_t launch_conv3x3_mfma_t(const View &in, const __bf16 *wp, const float *bias, const View &out, int N,
                                 int cin, int cout, int cin_pad, bool relu, bool vec, const View &pool,
                                 const View &up, hipStream_t s) {
    const int tiles = ((in.W + TWD - 1) / TWD) * ((in.H + MH - 1) / MH);
    const dim3 grid(tiles, N * ((cout + 16 * NM - 1) / (16 * NM)));
    const int r = relu ? 1 : 0, nt = ConvTile<TWD>::NT;
    if (vec)
        k_conv3x3_mfma<TO, NM, true, TWD><<<grid, nt, 0, s>>>(in, wp, bias, out, pool, up, cin, cout, cin_pad, r);
    else
        k_conv3x3_mfma<TO, NM, false, TWD><<<grid, nt, 0, s>>>(in, wp, bias, out, pool, up, cin, cout, cin_pad, r);
    return hipGetLastError();
}

// pool, up (may be NULL): the 2 x 2 pooled and the 2x upsampled output the
// epilogue also writes when the tile goes through LDS (*pooled, *upped set to
// whether it did).
template <class TO>
hipError_t launch_conv3x3_mfma(const View &in, const __bf16 *wp, const float *bias, const View &out, int N,
                               int cin, int cout, int cin_pad, bool relu, hipStream_t s,
                               const View *pool = nullptr, bool *pooled = nullptr, const View *up = nullptr,
                               bool *upped = nullptr) {
    const bool vec = mfma_vec_ok<TO>(in, out);
    View pv{};
    const bool fuse = pool != nullptr && vec && sizeof(TO) == 2 && in.H % 2 == 0 && in.W % 2 == 0 &&
                      2 * pool->H == in.H && 2 * pool->W == in.W && pool->W % 8 == 0 &&
                      ((long long)pool->H * pool->W) % 8 == 0 && pool->bs % 8 == 0 &&
                      (uintptr_t)pool->p % 16 == 0;
    if (fuse) pv = *pool;
    if (pooled) *pooled = fuse;
    View uv{};
    const bool fuse_up = up != nullptr && vec && sizeof(TO) == 2 && up->H == 2 * in.H && up->W == 2 * in.W &&
                         up->W % 16 == 0 && ((long long)up->H * up->W) % 8 == 0 && up->bs % 8 == 0 &&
                         (uintptr_t)up->p % 16 == 0;
    if (fuse_up) uv = *up;
    if (upped) *upped = fuse_up;
    const long long rows = (in.H + MH - 1) / MH;
    const bool narrow = mfma_narrow(cout) || rows * ((in.W + 31) / 32) * N * ((cout + 63) / 64) < 128;
    const long long wide_wgs = rows * (in.W / 64) * N * (narrow ? (cout + 31) / 32 : (cout + 63) / 64);
    const bool wide = vec && in.W % 64 == 0 && wide_wgs >= 256;
    if (narrow)
        return wide ? launch_conv3x3_mfma_t<TO, 2, 64>(in, wp, bias, out, N, cin, cout, cin_pad, relu, vec, pv, uv, s)
                    : launch_conv3x3_mfma_t<TO, 2, 32>(in, wp, bias, out, N, cin, cout, cin_pad, relu, vec, pv, uv, s);
    return wide ? launch_conv3x3_mfma_t<TO, 4, 64>(in, wp, bias, out, N, cin, cout, cin_pad, relu, vec, pv, uv, s)
                : launch_conv3x3_mfma_t<TO, 4, 32>(in, wp, bias, out, N, cin, cout, cin_pad, relu, vec, pv, uv, s);
}

hipError_t pack_all(const float *theta, __bf16 *base, const PackJobs &jobs, hipStream_t s) {
    if (jobs.n <= 0) return hipSuccess;
    if (jobs.n > PackJobs::MAX) return hipErrorInvalidValue;
    int most = 0;
    for (int k = 0; k < jobs.n; ++k) most = std::max(most, 9 * jobs.job[k].rows * jobs.job[k].pad);
    k_pack_all<<<dim3(std::min(nblk((size_t)most), 64u), (unsigned)jobs.n), 256, 0, s>>>(theta, base, jobs);
    return hipGetLastError();
}

hipError_t conv3x3_mfma_dx_packed(const View &dz, const __bf16 *wp, const View &dx, int N, int cin, int cout,
                                  hipStream_t s) {
    return launch_conv3x3_mfma<float>(dz, wp, nullptr, dx, N, cout, cin, pad32(cout), false, s);
}

hipError_t conv3x3_mfma_packed(const View &in, const __bf16 *wp, const float *bias, const View &out, int N,
                               int cin, int cout, bool relu, hipStream_t s, const View *pool, bool *pooled,
                               const View *up, bool *upped) {
    return launch_conv3x3_mfma<__bf16>(in, wp, bias, out, N, cin, cout, pad32(cin), relu, s, pool, pooled, up,
                                       upped);
}

hipError_t flip_transpose(const float *w, float *wt, int cin, int cout, hipStream_t s) {
    k_flip_transpose<<<nblk((size_t)cin * cout * 9), 256, 0, s>>>(w, wt, cin, cout);
    return hipGetLastError();
}

namespace {
// The first layer (at most four input planes) uses the 32 x 4 x 2 shape of
// k_conv3x3_dw, every other layer 16 x 16 x 1.
bool dw_small(int cin) { return cin <= 4; }

// Both gradient sums of a layer (k_sum_grads): OB = 64 outputs per workgroup
// when there are many, else 16 (more threads per output, fewer loads each).
hipError_t sum_grads(const float *partial, int chunks, int n, float *dw, const float *bpart, int nb, int C,
                     float *db, hipStream_t s) {
    if (!bpart) C = 0;
    if (n >= 64 * 512) {
        const int wb = (n + 63) / 64;
        k_sum_grads<64><<<wb + (C + 63) / 64, 256, 0, s>>>(partial, chunks, n, dw, bpart, nb, C, db, wb);
    } else {
        const int wb = (n + 15) / 16;
        k_sum_grads<16><<<wb + (C + 15) / 16, 256, 0, s>>>(partial, chunks, n, dw, bpart, nb, C, db, wb);
    }
    return hipGetLastError();
}
}  // namespace

int dw_chunks(int N, int H, int W, int cin, int cout) {
    const int ntiles = N * ((W + TW - 1) / TW) * ((H + TH - 1) / TH);
    if (dw_small(cin)) {
        // about 1024 workgroups of at least 2 tiles (256 workgroups of 8 tiles
        // measured 132 us at 64 x 256 x 32 samples: too few to hide the staging)
        const int blocks = (cout + 31) / 32;
        return std::max(1, std::min(ntiles / 2, (1024 + blocks - 1) / blocks));
    }
    const int blocks = ((cout + 15) / 16) * ((cin + 15) / 16);
    // aim for >= 2048 workgroups, at least 2 tiles per chunk
    return std::max(1, std::min(ntiles / 2, (2048 + blocks - 1) / blocks));
}

template <class TI>
hipError_t conv3x3_dw(const View &x, const float *dz, int N, int cin, int cout, float *partial, int chunks,
                      float *dw, const float *bpart, int nb, float *db, hipStream_t s) {
    const int ntiles = N * ((x.W + TW - 1) / TW) * ((x.H + TH - 1) / TH);
    const int per = (ntiles + chunks - 1) / chunks;
    if (dw_small(cin)) {
        const dim3 grid(chunks, (cout + 31) / 32, 1);
        k_conv3x3_dw<TI, 32, 4, 2><<<grid, 256, 0, s>>>(x, dz, N, cin, cout, per, partial);
    } else {
        const dim3 grid(chunks, (cout + 15) / 16, (cin + 15) / 16);
        k_conv3x3_dw<TI, 16, 16, 1><<<grid, 256, 0, s>>>(x, dz, N, cin, cout, per, partial);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sum_grads(partial, chunks, cout * cin * 9, dw, bpart, nb, cout, db, s);
}
template hipError_t conv3x3_dw<float>(const View &, const float *, int, int, int, float *, int, float *,
                                      const float *, int, float *, hipStream_t);
template hipError_t conv3x3_dw<__bf16>(const View &, const float *, int, int, int, float *, int, float *,
                                       const float *, int, float *, hipStream_t);

int dw_chunks_mfma(int N, int H, int W, int cin, int cout) {
    const int ntiles = N * ((W + DM_TW - 1) / DM_TW) * ((H + DM_TR - 1) / DM_TR);
    const int blocks = ((cout + DM_CO - 1) / DM_CO) * ((cin + DM_CI - 1) / DM_CI);
    // about 512 workgroups, at least 2 tiles per chunk: fewer chunk partials to
    // sum (training measured 3.75 ms per batch with 1024, 3.56 with 512, 3.74
    // with 256, with a one-thread-per-output sum)
    return std::max(1, std::min(ntiles / 2, (512 + blocks - 1) / blocks));
}

hipError_t conv3x3_dw_mfma(const View &x, const __bf16 *dz, int N, int cin, int cout, float *partial, int chunks,
                           float *dw, const float *bpart, int nb, float *db, hipStream_t s) {
    const int ntiles = N * ((x.W + DM_TW - 1) / DM_TW) * ((x.H + DM_TR - 1) / DM_TR);
    const int per = (ntiles + chunks - 1) / chunks;
    // vector staging: whole tile rows and 16-byte aligned rows of x and dz
    const size_t hw = (size_t)x.H * x.W;
    const int vec = x.W % DM_TW == 0 && hw % 8 == 0 && x.bs % 8 == 0 && (uintptr_t)x.p % 16 == 0 &&
                    (uintptr_t)dz % 16 == 0;
    const dim3 grid(chunks, (cout + DM_CO - 1) / DM_CO, (cin + DM_CI - 1) / DM_CI);
    if (vec) k_conv3x3_dw_mfma<true><<<grid, 256, 0, s>>>(x, dz, N, cin, cout, per, partial);
    else k_conv3x3_dw_mfma<false><<<grid, 256, 0, s>>>(x, dz, N, cin, cout, per, partial);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return sum_grads(partial, chunks, cout * cin * 9, dw, bpart, nb, cout, db, s);
}

namespace {
bool relu_vec4(const View &g, const View &y, const float *dz, const __bf16 *dzh) {
    const long long HW = (long long)y.H * y.W;
    return HW % 4 == 0 && g.bs % 4 == 0 && y.bs % 4 == 0 && (uintptr_t)g.p % 16 == 0 && (uintptr_t)y.p % 16 == 0 &&
           (uintptr_t)dz % 16 == 0 && (uintptr_t)dzh % 8 == 0;
}
}  // namespace

size_t bias_scratch(int N, int C, int H, int W) {
    return (size_t)N * C * nblk((size_t)H * W);   // the one-pixel-per-thread grid: the larger one
}

template <class TA>
hipError_t relu_mask_bias(const View &g, const View &y, int N, int C, float *dz, __bf16 *dzh, float *part,
                          int *nparts, hipStream_t s, const View *pool_g, const View *up_g) {
    const long long HW = (long long)y.H * y.W;
    const bool v4 = relu_vec4(g, y, dz, dzh);
    // the adjoint folded into the pass where its reads stay aligned (four fine
    // pixels of a row map to two pooled values, 8 bytes, or to two rows of
    // eight upsampled values, 2 x 32 bytes); otherwise it runs first, on g
    View pv{}, uv{};
    if (pool_g) {
        if (v4 && y.W % 4 == 0 && 2 * pool_g->H == y.H && 2 * pool_g->W == y.W && pool_g->W % 2 == 0 &&
            pool_g->bs % 2 == 0 && (uintptr_t)pool_g->p % 8 == 0) {
            pv = *pool_g;
        } else {
            const hipError_t e = pool_back_acc(*pool_g, g, N, C, s);
            if (e != hipSuccess) return e;
        }
    }
    if (up_g) {
        if (v4 && y.W % 4 == 0 && up_g->H == 2 * y.H && up_g->W == 2 * y.W && up_g->bs % 4 == 0 &&
            (uintptr_t)up_g->p % 16 == 0) {
            uv = *up_g;
        } else {
            const hipError_t e = up_back(*up_g, g, N, C, s);
            if (e != hipSuccess) return e;
        }
    }
    unsigned nb;
    if (v4) {
        nb = (unsigned)((HW / 4 + 255) / 256);
        k_relu_mask4<TA><<<dim3(nb, (unsigned)C, (unsigned)N), 256, 0, s>>>(g, y, N, C, dz, dzh, part, pv, uv);
    } else {
        const dim3 grid = pix_grid(y.H, y.W, C, N);
        nb = grid.x;
        k_relu_mask<TA><<<grid, 256, 0, s>>>(g, y, N, C, dz, dzh, part);
    }
    *nparts = (int)(nb * (unsigned)N);
    return hipGetLastError();
}
template hipError_t relu_mask_bias<float>(const View &, const View &, int, int, float *, __bf16 *, float *, int *,
                                          hipStream_t, const View *, const View *);
template hipError_t relu_mask_bias<__bf16>(const View &, const View &, int, int, float *, __bf16 *, float *, int *,
                                           hipStream_t, const View *, const View *);

template <class TA>
hipError_t pool(const View &in, const View &out, int N, int C, hipStream_t s) {
    k_pool<TA><<<pix_grid(out.H, out.W, C, N), 256, 0, s>>>(in, out, N, C);
    return hipGetLastError();
}
template hipError_t pool<float>(const View &, const View &, int, int, hipStream_t);
template hipError_t pool<__bf16>(const View &, const View &, int, int, hipStream_t);

hipError_t pool_back_acc(const View &dy, const View &dx, int N, int C, hipStream_t s) {
    const bool v4 = dx.W % 4 == 0 && dy.W * 2 == dx.W && dy.bs % 2 == 0 && dx.bs % 4 == 0 &&
                    (uintptr_t)dy.p % 16 == 0 && (uintptr_t)dx.p % 16 == 0;
    if (v4) {
        const dim3 grid((unsigned)(((size_t)dx.H * dx.W / 4 + 255) / 256), (unsigned)C, (unsigned)N);
        k_pool_back_acc4<<<grid, 256, 0, s>>>(dy, dx, N, C);
    } else {
        k_pool_back_acc<<<pix_grid(dx.H, dx.W, C, N), 256, 0, s>>>(dy, dx, N, C);
    }
    return hipGetLastError();
}

template <class TA>
hipError_t up(const View &in, const View &out, int N, int C, hipStream_t s) {
    const bool v4 = out.W % 4 == 0 && in.W * 2 == out.W && in.bs % 2 == 0 && out.bs % 4 == 0 &&
                    (uintptr_t)in.p % 16 == 0 && (uintptr_t)out.p % 16 == 0;
    if (v4) {
        const dim3 grid((unsigned)(((size_t)out.H * out.W / 4 + 255) / 256), (unsigned)C, (unsigned)N);
        k_up4<TA><<<grid, 256, 0, s>>>(in, out, N, C);
    } else {
        k_up<TA><<<pix_grid(out.H, out.W, C, N), 256, 0, s>>>(in, out, N, C);
    }
    return hipGetLastError();
}
template hipError_t up<float>(const View &, const View &, int, int, hipStream_t);
template hipError_t up<__bf16>(const View &, const View &, int, int, hipStream_t);

hipError_t up_back(const View &dy, const View &dx, int N, int C, hipStream_t s) {
    k_up_back<<<pix_grid(dx.H, dx.W, C, N), 256, 0, s>>>(dy, dx, N, C);
    return hipGetLastError();
}

template <class TA>
hipError_t conv1x1(const View &in, const float *w, const float *b, int N, int cin, int cout, float *out,
                   hipStream_t s) {
    k_conv1x1<TA><<<nblk((size_t)N * in.H * in.W), 256, 0, s>>>(in, w, b, N, cin, cout, out);
    return hipGetLastError();
}
template hipError_t conv1x1<float>(const View &, const float *, const float *, int, int, int, float *, hipStream_t);
template hipError_t conv1x1<__bf16>(const View &, const float *, const float *, int, int, int, float *, hipStream_t);

hipError_t conv1x1_dx(const float *g, const float *w, int N, int cin, int cout, int HW, const View &dx,
                      hipStream_t s) {
    k_conv1x1_dx<<<nblk((size_t)N * HW), 256, 0, s>>>(g, w, N, cin, cout, HW, dx);
    return hipGetLastError();
}

int conv1x1_dw_scratch(int cin, int cout) { return cout * (cin + 1) * BIAS_PARTS; }

template <class TA>
hipError_t conv1x1_dw(const View &x, const float *g, int N, int cin, int cout, float *part, float *dw, float *db,
                      hipStream_t s) {
    const int pairs = cout * (cin + 1);
    k_conv1x1_dw_partial<TA><<<dim3(pairs, BIAS_PARTS), 256, 0, s>>>(x, g, N, cin, cout, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_conv1x1_dw_final<<<nblk(pairs, 64), 64, 0, s>>>(part, cin, cout, dw, db);
    return hipGetLastError();
}
template hipError_t conv1x1_dw<float>(const View &, const float *, int, int, int, float *, float *, float *,
                                      hipStream_t);
template hipError_t conv1x1_dw<__bf16>(const View &, const float *, int, int, int, float *, float *, float *,
                                       hipStream_t);

constexpr int LOSS_BLOCKS = 256;
int loss_blocks() { return LOSS_BLOCKS; }

hipError_t loss_and_grad(const float *y, const float *t, const uint8_t *mask, int N, int C, int HW, double *part,
                         double *stats, float *g, hipStream_t s) {
    k_loss_partial<<<LOSS_BLOCKS, 256, 0, s>>>(y, t, mask, N, C, HW, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_loss_final<<<1, 64, 0, s>>>(part, LOSS_BLOCKS, stats);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (g) k_loss_grad<<<nblk((size_t)N * C * HW), 256, 0, s>>>(y, t, mask, N, C, HW, stats, g);
    return hipGetLastError();
}

hipError_t adam(float *th, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s) {
    k_adam<<<nblk(n), 256, 0, s>>>(th, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t zero(float *p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_zero<<<(unsigned)std::min<size_t>(4096, nblk(n)), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

}  // namespace lbmnet
