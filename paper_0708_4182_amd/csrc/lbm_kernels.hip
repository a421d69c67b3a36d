// HIP kernels of the EWOD Shan-Chen D2Q9 lattice Boltzmann step for gfx950.
//
// Data layout: populations in structure-of-arrays planes [9][ny][pitch] (x
// fastest, pitch a multiple of 64 elements), double-buffered.  A buffer holds
// the post-collision populations f* of the last step; a step pulls
// f_a(x) = f*_a(x - e_a) (or the bounce-back f*_opp(a)(x) when x - e_a is solid),
// which is the streaming half of eq. (1), then collides.
//
// Velocity numbering (as in the paper): e_0 = (0,0); e_1..e_4 = (1,0), (0,1),
// (-1,0), (0,-1); e_5..e_8 = (1,1), (-1,1), (-1,-1), (1,-1).
#include "lbm_internal.h"

#include <algorithm>
#include <type_traits>

namespace lbm {
namespace {

enum { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2 };

typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Storage codecs.  Every format stores d = f - w_a rho_off (rho_off = 0 keeps
// f itself), FP16/BF16 rounded to nearest even by the hardware conversion.
template <int S> struct Codec;
template <> struct Codec<ST_F32> {
    using T = float;
    __device__ static float dec(T v) { return v; }
    __device__ static T enc(float v) { return v; }
};
template <> struct Codec<ST_F16> {
    using T = _Float16;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float v) { return (_Float16)v; }
    // Stochastic rounding with random bits r (low 13 used) by gfx950's
    // v_cvt_sr_f16_f32, which takes its random bits from the top of its second
    // operand: the magnitude rounds up with probability (dropped part) / (last
    // place of the result), so the expected result is v.  For FP16 normals the
    // 13 bits are added at the top of the 13-bit dropped field and the word is
    // truncated; in the FP16 subnormal range (last place 2^-24) the field is
    // longer and the 13 bits sit at its top (probabilities resolved to
    // 2^-13); below 2^-24 the result is 0 or 2^-24.  Inf and NaN convert as
    // they are, so a diverged node stays visible to the density guard.
    // (Checked on the device against that definition written out with
    // integer operations: bit-identical for every |v| >= 2^-24.)
    __device__ static T enc_sr(float v, uint32_t r) {
        const f16x2 z = {(_Float16)0.f, (_Float16)0.f};
        return __builtin_amdgcn_cvt_sr_f16_f32(z, v, r << 19, false)[0];
    }
};
template <> struct Codec<ST_BF16> {
    using T = __bf16;
    __device__ static float dec(T v) { return (float)v; }
    __device__ static T enc(float v) { return (__bf16)v; }
    // Stochastic rounding with random bits r (low 16 used) by gfx950's
    // v_cvt_sr_bf16_f32 (random bits from the top of its second operand): BF16
    // keeps the top 16 bits of the FP32 word, so the 16 random bits are added
    // to the whole dropped field and the word truncated (exactly unbiased);
    // Inf and NaN convert as they are.  (Bit-identical on the device to that
    // definition written out with integer operations.)
    __device__ static T enc_sr(float v, uint32_t r) {
        const bf16x2 z = {(__bf16)0.f, (__bf16)0.f};
        return __builtin_amdgcn_cvt_sr_bf16_f32(z, v, r << 16, false)[0];
    }
};

// 32-bit integer hash "lowbias32" (C. Wellons, hash-prospector: xor-shift 16,
// multiply, xor-shift 15, multiply, xor-shift 16).  Counter-based random bits
// for stochastic rounding: input = (node offset * 5 + k) xor a per-step mix.
__device__ __forceinline__ uint32_t lowbias32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

// Per-step random-bit mix of a stochastic-rounding step kernel.  The step
// count lives in a two-slot device counter: the kernel reads slot par (its
// source-buffer parity) and one lane of workgroup 0 writes count + 1 to the
// other slot, which only the next step reads.  The count therefore advances
// across hipGraph replays as across eager launches.
__device__ __forceinline__ uint32_t sr_step_mix(uint32_t *rng, int par) {
    const uint32_t count = rng[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) rng[par ^ 1] = count + 1u;
    return lowbias32(count + 0x9e3779b9u);
}

constexpr float W0 = 4.f / 9.f, W1 = 1.f / 9.f, W5 = 1.f / 36.f;

// Element access by 32-bit element offset from the buffer base; the offsets
// of one buffer stay below 2^32 bytes (checked by the host), so the address
// is base + zero-extended byte offset.
template <class T>
__device__ __forceinline__ T ld(const T *__restrict__ base, uint32_t off) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + off * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st(T *__restrict__ base, uint32_t off, T v) {
#ifdef LBM_NT_STORES
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off * (uint32_t)sizeof(T)));
#else
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + off * (uint32_t)sizeof(T)) = v;
#endif
}

// Buffer-resource access (raw buffer instructions): per-lane byte offset in a
// VGPR plus a wave-uniform byte offset in an SGPR.  The resource covers the
// whole buffer (< 4 GiB, checked by the host); reads outside it return 0.
constexpr int kBufWord3 = 0x00020000;   // gfx9-family raw buffer, 32-bit data
constexpr int kStoreNT = 2;             // non-temporal store (streamed output)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kBufWord3);
}
template <class T> __device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff);
template <> __device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ _Float16 bload<_Float16>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ __bf16 bload<__bf16>(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ uint32_t bload_flag(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return (uint32_t)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, kStoreNT);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, _Float16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)voff, (int)soff, kStoreNT);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, __bf16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, v), r, (int)voff, (int)soff, kStoreNT);
}

// Source offsets of the nine populations of node x under streaming with
// halfway bounce-back (pull form).  fl holds the neighbour solid bits of x:
// bit (b-1) = S(x + e_b).  Population a comes from x - e_a = x + e_opp(a); if
// that node is solid it is the post-collision population opp(a) of x itself.
// rm/r0/rp: element offsets of rows y-1, y, y+1; xm/x/xp: columns x-1, x, x+1
// (periodic).
__device__ __forceinline__ void pull_offsets(uint32_t fl, uint32_t plane, uint32_t rm, uint32_t r0,
                                             uint32_t rp, uint32_t xm, uint32_t x, uint32_t xp,
                                             uint32_t o[9]) {
    const uint32_t own = r0 + x;
    o[0] = own;
    o[1] = (fl & 0x04u) ? 3u * plane + own : 1u * plane + r0 + xm;   // from x-1     (e_3 side)
    o[2] = (fl & 0x08u) ? 4u * plane + own : 2u * plane + rm + x;    // from y-1     (e_4 side)
    o[3] = (fl & 0x01u) ? 1u * plane + own : 3u * plane + r0 + xp;   // from x+1     (e_1 side)
    o[4] = (fl & 0x02u) ? 2u * plane + own : 4u * plane + rp + x;    // from y+1     (e_2 side)
    o[5] = (fl & 0x40u) ? 7u * plane + own : 5u * plane + rm + xm;   // from (-1,-1) (e_7 side)
    o[6] = (fl & 0x80u) ? 8u * plane + own : 6u * plane + rm + xp;   // from (+1,-1) (e_8 side)
    o[7] = (fl & 0x10u) ? 5u * plane + own : 7u * plane + rp + xp;   // from (+1,+1) (e_5 side)
    o[8] = (fl & 0x20u) ? 6u * plane + own : 8u * plane + rp + xm;   // from (-1,+1) (e_6 side)
}

template <class C>
__device__ __forceinline__ void pull9(const typename C::T *__restrict__ src, uint32_t plane,
                                      uint32_t fl, uint32_t rm, uint32_t r0, uint32_t rp,
                                      uint32_t xm, uint32_t x, uint32_t xp, float d[9]) {
    uint32_t o[9];
    pull_offsets(fl, plane, rm, r0, rp, xm, x, xp, o);
#pragma unroll
    for (int a = 0; a < 9; ++a) d[a] = C::dec(ld(src, o[a]));
}

// eq. (2) on decoded values: s = sum d (= rho - rho_off), j = sum d e.  The
// rest offsets w_a rho_off of the stored deviations sum to rho_off and carry no momentum.
__device__ __forceinline__ void moments9(const float d[9], float &s, float &jx, float &jy) {
    s = (((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7]))) + d[8];
    jx = (d[1] - d[3]) + ((d[5] - d[7]) + (d[8] - d[6]));
    jy = (d[2] - d[4]) + ((d[5] - d[7]) + (d[6] - d[8]));
}

// eq. (4): psi = rho0 (1 - exp(-x)), x = rho / rho0.  In the vapour (x ~ 0.05)
// 1 - exp(-x) cancels about four bits of exp(-x), so it is evaluated as
// -expm1(-x) in W. Kahan's form: with t = -x log2(e) and u = 2^t (the hardware's
// base-2 exponential), expm1 = (u - 1) t / log2(u); the rounding error of u
// appears in both factors and cancels, which keeps psi to a few ulp at any x.
// u == 1 (|t| below half an ulp of 1) leaves the first-order term t ln 2.
__device__ __forceinline__ float pseudopotential(const Model &m, float rho) {
    const float t = -rho * m.log2e_inv_rho0;
    const float u = __builtin_amdgcn_exp2f(t);
    const float em1 = u == 1.f ? t * 0.693147180559945309f
                               : (u - 1.f) * (t * __builtin_amdgcn_rcpf(__builtin_amdgcn_logf(u)));
    return -m.rho0 * em1;
}

// f^eq of eq. (3) minus the stored rest offset w_a rho_off, for density rho
// (= rho_off + s) and momentum (jx, jy) = rho u.  Arranged so that the zeroth
// and first moments hold up to unbiased rounding even though 1/9 and 1/36 are
// not representable: the second-order part E of each opposite pair, the rest
// population as the remainder of the mass s, and the odd parts of the axis
// pairs as the remainder of the momentum.  In exact arithmetic this is eq. (3).
// Contraction into FMAs is off here: fusing 4.5 u_x u_x against the separately
// rounded u^2 breaks the consistency of the rounded second-order terms, and the
// resulting stress bias accumulates in slow near-wall films (measured: FP32
// results drift from FP64 by 1.6e-5 over 700 steps with contraction, 1.2e-6
// without).
__device__ __forceinline__ void equilibrium(float rho, float s, float jx, float jy, float feq[9]) {
#pragma clang fp contract(off)
    const float inv = __builtin_amdgcn_rcpf(rho);
    const float ux = jx * inv, uy = jy * inv;
    const float usq = 1.5f * (ux * ux + uy * uy);
    const float a = ux + uy, b = uy - ux;
    const float E1 = W1 * (s + rho * (4.5f * ux * ux - usq));
    const float E2 = W1 * (s + rho * (4.5f * uy * uy - usq));
    const float E5 = W5 * (s + rho * (4.5f * a * a - usq));
    const float E6 = W5 * (s + rho * (4.5f * b * b - usq));
    const float E0 = s - 2.f * ((E1 + E2) + (E5 + E6));
    const float O5 = (jx + jy) * (1.f / 12.f);
    const float O6 = (jy - jx) * (1.f / 12.f);
    const float O1 = 0.5f * jx - (O5 - O6);
    const float O2 = 0.5f * jy - (O5 + O6);
    feq[0] = E0;
    feq[1] = E1 + O1;
    feq[3] = E1 - O1;
    feq[2] = E2 + O2;
    feq[4] = E2 - O2;
    feq[5] = E5 + O5;
    feq[7] = E5 - O5;
    feq[6] = E6 + O6;
    feq[8] = E6 - O6;
}

// Two-relaxation-time collision with Guo's forcing term (lbm_params.collision
// = LBM_COLLIDE_TRT_GUO; not the paper's scheme).  The equilibrium and the
// source take u = (j + F/2) / rho; each opposite pair (a, b) relaxes its
// symmetric part n+ = ((f - feq)_a + (f - feq)_b) / 2 at omega+ and its
// antisymmetric part n- at omega-, and gets the matching parts of
// S_a = w_a [3 (e_a - u) . F + 9 (e_a . u)(e_a . F)]:
// S+ = w (9 (e.u)(e.F) - 3 u.F) weighted 1 - omega+/2, S- = 3 w e.F weighted
// 1 - omega-/2.  Deviations d and feq share the offset w rho_off, which
// cancels in n+ and n-.
__device__ __forceinline__ void collide_trt(const Model &m, const float d[9], float rho, float s, float jx,
                                            float jy, float Fx, float Fy, float out[9]) {
#pragma clang fp contract(off)
    const float hx = jx + 0.5f * Fx, hy = jy + 0.5f * Fy;
    float feq[9];
    equilibrium(rho, s, hx, hy, feq);
    const float inv = __builtin_amdgcn_rcpf(rho);
    const float ux = hx * inv, uy = hy * inv;
    const float uF3 = 3.f * (ux * Fx + uy * Fy);
    const float wp = m.omega, wm = m.omega_m, cp = m.src_p, cm = m.src_m;
    out[0] = d[0] - wp * (d[0] - feq[0]) - cp * (W0 * uF3);
    auto pair = [&](int a, int b, float eu, float eF, float w) {
        const float na = d[a] - feq[a], nb = d[b] - feq[b];
        const float np = 0.5f * (na + nb), nm = 0.5f * (na - nb);
        const float sp = w * (9.f * eu * eF - uF3), sm = 3.f * w * eF;
        const float sym = cp * sp - wp * np, anti = cm * sm - wm * nm;
        out[a] = d[a] + (sym + anti);
        out[b] = d[b] + (sym - anti);
    };
    pair(1, 3, ux, Fx, W1);
    pair(2, 4, uy, Fy, W1);
    pair(5, 7, ux + uy, Fx + Fy, W5);
    pair(6, 8, uy - ux, Fy - Fx, W5);
}

// Multiple-relaxation-time collision with Guo's forcing term
// (lbm_params.collision = LBM_COLLIDE_MRT_GUO; not the paper's scheme), run
// by the TRT kernels.  The non-equilibrium parts n = d - feq (feq at
// u = (j + F/2) / rho, the offset w rho_off cancelling as in TRT) go to the
// six non-conserved moments of the orthogonal basis (e, eps, q_x, q_y, p_xx,
// p_xy), built from the sums P and differences D of opposite pairs; each
// relaxes at its rate and gets (1 - s/2) times its moment of Guo's source,
// which in this basis is (6 u.F, -6 u.F, -F_x, -F_y, 2 (u_x F_x - u_y F_y),
// u_x F_y + u_y F_x); j gains F, rho nothing.  The changes go back through
// M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4).
__device__ __forceinline__ void collide_mrt(const Model &m, const float d[9], float rho, float s, float jx,
                                            float jy, float Fx, float Fy, float out[9]) {
#pragma clang fp contract(off)
    const float hx = jx + 0.5f * Fx, hy = jy + 0.5f * Fy;
    float feq[9];
    equilibrium(rho, s, hx, hy, feq);
    const float inv = __builtin_amdgcn_rcpf(rho);
    const float ux = hx * inv, uy = hy * inv;
    float n[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) n[a] = d[a] - feq[a];
    const float P1 = n[1] + n[3], D1 = n[1] - n[3], P2 = n[2] + n[4], D2 = n[2] - n[4];
    const float P5 = n[5] + n[7], D5 = n[5] - n[7], P6 = n[6] + n[8], D6 = n[6] - n[8];
    const float ne = 2.f * (P5 + P6) - (P1 + P2) - 4.f * n[0];
    const float neps = (P5 + P6) - 2.f * (P1 + P2) + 4.f * n[0];
    const float nqx = (D5 - D6) - 2.f * D1, nqy = (D5 + D6) - 2.f * D2;
    const float npxx = P1 - P2, npxy = P5 - P6;
    const float se = m.mrt_se, seps = m.mrt_seps, sq = m.omega_m, sn = m.omega;
    const float uF = ux * Fx + uy * Fy;
    const float de = (1.f - 0.5f * se) * (6.f * uF) - se * ne;
    const float deps = (1.f - 0.5f * seps) * (-6.f * uF) - seps * neps;
    const float dqx = (1.f - 0.5f * sq) * (-Fx) - sq * nqx;
    const float dqy = (1.f - 0.5f * sq) * (-Fy) - sq * nqy;
    const float dpxx = (1.f - 0.5f * sn) * (2.f * (ux * Fx - uy * Fy)) - sn * npxx;
    const float dpxy = (1.f - 0.5f * sn) * (ux * Fy + uy * Fx) - sn * npxy;
    const float ce = de * (1.f / 36.f), cp = deps * (1.f / 36.f);
    const float cjx = Fx * (1.f / 6.f), cjy = Fy * (1.f / 6.f);
    const float cqx = dqx * (1.f / 12.f), cqy = dqy * (1.f / 12.f);
    const float cxx = 0.25f * dpxx, cxy = 0.25f * dpxy;
    const float ax = -ce - 2.f * cp;              // even part shared by the axis directions
    const float dg = 2.f * ce + cp;               // and by the diagonals
    const float ox = cjx - 2.f * cqx, oy = cjy - 2.f * cqy;
    const float gx = cjx + cqx, gy = cjy + cqy;
    out[0] = d[0] + 4.f * (cp - ce);
    out[1] = d[1] + ((ax + cxx) + ox);
    out[3] = d[3] + ((ax + cxx) - ox);
    out[2] = d[2] + ((ax - cxx) + oy);
    out[4] = d[4] + ((ax - cxx) - oy);
    out[5] = d[5] + ((dg + cxy) + (gx + gy));
    out[7] = d[7] + ((dg + cxy) - (gx + gy));
    out[6] = d[6] + ((dg - cxy) + (gy - gx));
    out[8] = d[8] + ((dg - cxy) - (gy - gx));
}

// Force, velocity shift (eq. (10)) and BGK collision (eq. (1)) of one node,
// then the store of its nine post-collision populations.  phi of the 3x3
// neighbourhood comes from LDS rows rowm (y-1), row0 (y), rowp (y+1) at
// column c; solid neighbours hold phi = 0 there, which removes them from
// eq. (5) as the model requires.
template <bool TRT>
__device__ __forceinline__ void collide_post(const Model &m, const float d[9], float s, float jx, float jy,
                                             uint32_t fl, const float *rowm, const float *row0,
                                             const float *rowp, int c, float out[9]) {
    const float rho = m.rho_off + s;
    const float pc = row0[c];
    const float p1 = row0[c + 1], p3 = row0[c - 1];
    const float p2 = rowp[c], p4 = rowm[c];
    const float p5 = rowp[c + 1], p6 = rowp[c - 1], p7 = rowm[c - 1], p8 = rowm[c + 1];
    // eq. (5)
    float sx = m.ga * (p1 - p3) + m.gd * ((p5 - p7) + (p8 - p6));
    float sy = m.ga * (p2 - p4) + m.gd * ((p5 - p7) + (p6 - p8));
    // eq. (6): S(x + e_b) = bit (b-1) of fl
    if (fl & 0xFFu) {
        const float s1 = (float)(fl & 1u), s2 = (float)((fl >> 1) & 1u), s3 = (float)((fl >> 2) & 1u),
                    s4 = (float)((fl >> 3) & 1u), s5 = (float)((fl >> 4) & 1u), s6 = (float)((fl >> 5) & 1u),
                    s7 = (float)((fl >> 6) & 1u), s8 = (float)((fl >> 7) & 1u);
        sx += m.wa * (s1 - s3) + m.wd * ((s5 - s7) + (s8 - s6));
        sy += m.wa * (s2 - s4) + m.wd * ((s5 - s7) + (s6 - s8));
    }
    float Fx = -pc * sx, Fy = -pc * sy;
    // electric force on the conductive part of the layer, n towards the electrode
    if ((fl & FL_LAYER) && rho >= m.rho_c) {
        const uint32_t a = (fl >> FL_NSHIFT) & 15u;
        if (a == 0u) {
            Fy += (fl & FL_TOP) ? m.f_elec : -m.f_elec;
        } else {   // along e_a / |e_a|; e_x + 1, e_y + 1 packed in 2 bits per direction
            const float fa = a >= 5u ? m.f_elec_diag : m.f_elec;
            Fx += fa * (float)((int)((0x20919u >> (2u * a)) & 3u) - 1);
            Fy += fa * (float)((int)((0x02865u >> (2u * a)) & 3u) - 1);
        }
    }
    // driving body force
    Fx += rho * m.gx;
    Fy += rho * m.gy;
    if constexpr (TRT) {
        if (m.trt == 2) collide_mrt(m, d, rho, s, jx, jy, Fx, Fy, out);
        else collide_trt(m, d, rho, s, jx, jy, Fx, Fy, out);
        return;
    }
    // eq. (10): rho u' = rho u + tau F
    float feq[9];
    equilibrium(rho, s, jx + m.tau * Fx, jy + m.tau * Fy, feq);
    const float om = m.omega;
#pragma unroll
    for (int a = 0; a < 9; ++a) out[a] = d[a] + om * (feq[a] - d[a]);
}

// The collision with its nine results encoded for storage (nearest).
template <class C, bool TRT = false>
__device__ __forceinline__ void collide(const Model &m, const float d[9], float s, float jx, float jy,
                                        uint32_t fl, const float *rowm, const float *row0,
                                        const float *rowp, int c, typename C::T out[9]) {
    float p[9];
    collide_post<TRT>(m, d, s, jx, jy, fl, rowm, row0, rowp, c, p);
#pragma unroll
    for (int a = 0; a < 9; ++a) out[a] = C::enc(p[a]);
}

// With SR the nine results are rounded stochastically: 16 random bits each,
// from five hashes of (node offset * 5 + k) xor the step's mix.
template <class C, bool TRT = false, bool SR = false>
__device__ __forceinline__ void collide_store(const Model &m, const float d[9], float s, float jx,
                                              float jy, uint32_t fl, const float *rowm,
                                              const float *row0, const float *rowp, int c,
                                              __amdgpu_buffer_rsrc_t dst, uint32_t plane,
                                              uint32_t row, uint32_t lane_byte, uint32_t mix = 0u) {
    constexpr uint32_t E = sizeof(typename C::T);
    typename C::T out[9];
    if constexpr (SR) {
        float p[9];
        collide_post<TRT>(m, d, s, jx, jy, fl, rowm, row0, rowp, c, p);
        const uint32_t k0 = (row + lane_byte / E) * 5u;
        uint32_t h[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) h[k] = lowbias32((k0 + (uint32_t)k) ^ mix);
#pragma unroll
        for (int a = 0; a < 9; ++a) out[a] = C::enc_sr(p[a], (a & 1) ? (h[a >> 1] >> 16) : (h[a >> 1] & 0xFFFFu));
    } else {
        collide<C, TRT>(m, d, s, jx, jy, fl, rowm, row0, rowp, c, out);
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) bstore(dst, lane_byte, ((uint32_t)a * plane + row) * E, out[a]);
}

// Barrier that orders LDS only; global loads in flight are not waited for.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Per-direction constants for the halo gather.
__constant__ int8_t kEX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__constant__ int8_t kEY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
__constant__ int8_t kOPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
// neighbour bit of x - e_a (= bit of opp(a) - 1); none for the rest population
__constant__ uint16_t kSRCBIT[9] = {0, 0x04, 0x08, 0x01, 0x02, 0x40, 0x80, 0x10, 0x20};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Fused step.  A workgroup of BX threads owns the columns [x0, x0 + BX) of one
// strip and marches through the rows [y0, y1) of one chunk, upwards for even
// chunks and downwards for odd ones (so that two chunks read their shared
// halo rows at about the same time).  For each pulled row it computes rho and
// phi (one node per thread) and puts phi in a 4-row LDS ring that carries one
// halo column on each side; after one barrier it collides the previous row,
// whose phi neighbourhood is then complete.  The flag word of a row is loaded
// two rows ahead and its populations one row ahead, with the bounce-back
// addresses already resolved, so HBM latency overlaps the collision.  The halo
// columns are gathered by 18 lanes of wave 0 (one population each) and
// reduced with lane shuffles.  Workgroups map to tiles so that consecutive
// chunks of a strip run on the same XCD.
constexpr int RING = 4;

// EXT: a per-node acceleration field acc [2][ny][nx] (x plane, then y plane;
// dense rows of nx) is added to the driving acceleration of each node.
template <int S, bool TRT = false, bool SR = false, bool EXT = false>
__device__ __forceinline__ void step_tile(const void *src_ptr, void *dst_ptr, const uint16_t *flags_ptr,
                                          const uint32_t *__restrict__ rowplain, const Grid &g, const Model &m,
                                          int x0, int y0, int y1, bool up, float *ring, uint32_t mix = 0u,
                                          const float *__restrict__ acc = nullptr) {
    using C = Codec<S>;
    using T = typename C::T;
    const int BX = blockDim.x, W = BX + 2;
    const int tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny;
    const uint32_t pitch = (uint32_t)g.pitch, plane = g.plane;
    constexpr uint32_t E = sizeof(T);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src_ptr, 9u * plane * E);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst_ptr, 9u * plane * E);
    const __amdgpu_buffer_rsrc_t rf = make_rsrc(flags_ptr, plane * 2u);
    const int nrows = y1 - y0 + 2;      // pulled rows: the chunk plus one halo row per side

    const int nact = min(BX, nx - x0);
    const bool act = tid < nact;
    const int x = x0 + (act ? tid : 0);
    const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;

    // halo gather lanes: 0..8 left column, 16..24 right column, one population
    // each; lanes of wave 0 outside the gather take population 0.  Their
    // addressing is recomputed per row (wave 0 only) from a copy of the thread
    // index the compiler cannot see through, so that it is not held in
    // registers of every wave through the collision.
    const bool hlane = tid < 32 && (tid & 15) < 9;
    auto opaque = [](int v) {
        asm volatile("" : "+v"(v));
        return v;
    };
    auto halo_x = [&](int t) { return (t < 16) ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + nact == nx ? 0 : x0 + nact); };

    auto row_at = [&](int i) {
        const int r = up ? y0 - 1 + i : y1 - i;
        return wrapi(r, ny);
    };

    // pipeline registers
    uint32_t fl1 = FL_SOLID, fl2 = FL_SOLID, hfl1 = FL_SOLID, hfl2 = FL_SOLID;   // rows i+1, i+2
    T raw[9];
    T hraw = C::enc(0.f);
    float pd[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float ps = 0.f, pjx = 0.f, pjy = 0.f;
    uint32_t pfl = FL_SOLID;
    int pyr = 0;

    // Every lane loads (no per-lane branches): inactive lanes use the clamped
    // column x0, solid nodes have no neighbour bits and read their (wrapped)
    // neighbours, and lanes of wave 0 outside the halo gather read population 0
    // of a halo node, so every address is inside the buffer.  Those values are
    // discarded.
    // A wave whose columns do not wrap around x and none of whose nodes in the
    // row has a solid neighbour takes the fast path: byte offsets of columns
    // x-1, x, x+1 are loop invariants and plane and row go into the scalar
    // offset, so the nine loads need no address arithmetic.
    const int wave_x0 = x0 + (tid & ~63);
    const bool wave_wraps = wave_x0 == 0 || wave_x0 + 64 > nx - 1;
    const uint32_t v0 = (uint32_t)x * E, vm = xm * E, vp = xp * E;
    const uint32_t vf = (uint32_t)x * 2u;
    auto issue_pops = [&](int yr, uint32_t fl, uint32_t hfl) {
        const int ym = yr == 0 ? ny - 1 : yr - 1, yp = yr == ny - 1 ? 0 : yr + 1;
        const uint32_t r0 = (uint32_t)yr * pitch, rm = (uint32_t)ym * pitch, rp = (uint32_t)yp * pitch;
        if (!wave_wraps && __builtin_amdgcn_ballot_w64((fl & 0xFFu) != 0u) == 0) {
            raw[0] = bload<T>(rs, v0, (0u * plane + r0) * E);
            raw[1] = bload<T>(rs, vm, (1u * plane + r0) * E);
            raw[2] = bload<T>(rs, v0, (2u * plane + rm) * E);
            raw[3] = bload<T>(rs, vp, (3u * plane + r0) * E);
            raw[4] = bload<T>(rs, v0, (4u * plane + rp) * E);
            raw[5] = bload<T>(rs, vm, (5u * plane + rm) * E);
            raw[6] = bload<T>(rs, vp, (6u * plane + rm) * E);
            raw[7] = bload<T>(rs, vp, (7u * plane + rp) * E);
            raw[8] = bload<T>(rs, vm, (8u * plane + rp) * E);
        } else {
            uint32_t o[9];
            pull_offsets(fl & 0xFFu, plane, rm, r0, rp, xm, (uint32_t)x, xp, o);
#pragma unroll
            for (int q = 0; q < 9; ++q) raw[q] = bload<T>(rs, o[q] * E, 0u);
        }
        if (tid < 64) {
            // e_a and opp(a) of the gathered population a from packed tables:
            // e_x + 1 and e_y + 1 in 2 bits, opp(a) in 4 bits per direction
            const int t = opaque(tid);
            const int ha = (t < 32 && (t & 15) < 9) ? (t & 15) : 0;
            const int hx = halo_x(t);
            const int ex = (int)((0x20919u >> (2 * ha)) & 3u) - 1;
            const int ey = (int)((0x02865u >> (2 * ha)) & 3u) - 1;
            const uint32_t opp = (uint32_t)((0x658721430ull >> (4 * ha)) & 15u);
            const uint32_t srcbit = ha == 0 ? 0u : 1u << (opp - 1u);    // bit of x - e_a
            const uint32_t hsx = (uint32_t)wrapi(hx - ex, nx);
            const uint32_t hrow = ey > 0 ? rm : (ey < 0 ? rp : r0);   // row of y - e_y
            const uint32_t off = (hfl & srcbit) ? opp * plane + r0 + (uint32_t)hx
                                                : (uint32_t)ha * plane + hrow + hsx;
            hraw = bload<T>(rs, off * E, 0u);
        }
    };
    // FP32 storage: a row whose nodes all carry the plain flag word (fluid,
    // no solid neighbour, outside the electric layer: 0, or FL_TOP in the top
    // half) takes it from the row's bit instead of loading its flags (2 of
    // the 74 bytes per node).  The bits of the 128 rows from the word holding
    // row y0 - 1 are read once per tile into uniform registers, so the test
    // per row is scalar arithmetic with no wait; rows outside that window,
    // and the halo rows that wrap around the lattice, load their flags.  The
    // 16-bit kernels measured no faster with it and keep the plain loads.
    constexpr bool ROWBITS = S == ST_F32;
    const int ubase = max(y0 - 1, 0) & ~31;
    uint64_t plo = 0, phi = 0;
    if constexpr (ROWBITS) {
        const uint32_t nwords = ((uint32_t)ny + 31u) >> 5, w0 = (uint32_t)ubase >> 5;
        uint32_t w[4];
#pragma unroll
        for (uint32_t k = 0; k < 4; ++k) w[k] = w0 + k < nwords ? rowplain[w0 + k] : 0u;
        plo = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
        phi = (uint64_t)w[2] | ((uint64_t)w[3] << 32);
    }
    auto issue_flags = [&](int i, int yr, uint32_t &fl, uint32_t &hfl) {
        if constexpr (ROWBITS) {
            const int u = up ? y0 - 1 + i : y1 - i;   // the row before wrapping
            const int d = u - ubase;
            const bool plain = u >= 0 && u < ny && d >= 0 && d < 128 &&
                               ((d < 64 ? plo >> d : phi >> (d - 64)) & 1u);   // uniform for the workgroup
            if (plain) {
                const uint32_t v = yr >= (ny >> 1) ? FL_TOP : 0u;
                fl = v;
                if (tid < 64) hfl = v;
                return;
            }
        }
        const uint32_t r0b = (uint32_t)yr * pitch * 2u;
        fl = bload_flag(rf, vf, r0b);
        if (tid < 64) hfl = bload_flag(rf, (uint32_t)halo_x(opaque(tid)) * 2u, r0b);
    };

    // prologue: flags of rows 0 and 1, populations of row 0
    {
        uint32_t f0 = FL_SOLID, h0 = FL_SOLID;
        issue_flags(0, row_at(0), f0, h0);
        issue_flags(1, row_at(1), fl2, hfl2);
        issue_pops(row_at(0), f0, h0);
        fl1 = f0;
        hfl1 = h0;
    }

    for (int i = 0; i < nrows; ++i) {
        const int yr = row_at(i);
        // take row i from the pipeline and start rows i+1 (populations) and i+2 (flags)
        const uint32_t cfl = fl1, chfl = hfl1;
        T craw[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) craw[q] = raw[q];
        const T chraw = hraw;
        fl1 = fl2;
        hfl1 = hfl2;
        // past the end of the chunk the last row is fetched again (cache hits),
        // which keeps the pipeline free of branches
        issue_flags(min(i + 2, nrows - 1), row_at(min(i + 2, nrows - 1)), fl2, hfl2);
        issue_pops(row_at(min(i + 1, nrows - 1)), fl1, hfl1);

        float *slot = ring + (i & (RING - 1)) * W;
        float cd[9], cs = 0.f, cjx = 0.f, cjy = 0.f;
#pragma unroll
        for (int q = 0; q < 9; ++q) cd[q] = C::dec(craw[q]);
        moments9(cd, cs, cjx, cjy);
        if (act) slot[tid + 1] = (cfl & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + cs);
        if (tid < 64) {
            // rho of the two halo nodes, summed in the same order as moments9 so
            // that a column gets bitwise the same phi as a halo or as an own node
            const float hv = (hlane && !(chfl & FL_SOLID)) ? C::dec(chraw) : 0.f;
            const int base = tid & ~15;
            float g[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) g[q] = __shfl(hv, base + q, 64);
            if (tid == 0 || tid == 16) {
                const float hs = (((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7]))) + g[8];
                const float phi = (chfl & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + hs);
                slot[tid == 0 ? 0 : nact + 1] = phi;
            }
        }
        lds_barrier();
        if (i >= 2 && act && !(pfl & FL_SOLID)) {
            const float *older = ring + ((i - 2) & (RING - 1)) * W;
            const float *mid = ring + ((i - 1) & (RING - 1)) * W;
            const float *rowm = up ? older : slot;
            const float *rowp = up ? slot : older;
            if constexpr (EXT) {
                // the node's acceleration joins the uniform one: rho (g + acc)
                const size_t k = (size_t)pyr * (size_t)nx + (size_t)x;
                Model mx = m;
                mx.gx = m.gx + acc[k];
                mx.gy = m.gy + acc[(size_t)nx * (size_t)ny + k];
                collide_store<C, TRT, SR>(mx, pd, ps, pjx, pjy, pfl, rowm, mid, rowp, tid + 1, rd, plane,
                                          (uint32_t)pyr * pitch, v0, mix);
            } else {
                collide_store<C, TRT, SR>(m, pd, ps, pjx, pjy, pfl, rowm, mid, rowp, tid + 1, rd, plane,
                                          (uint32_t)pyr * pitch, v0, mix);
            }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) pd[q] = cd[q];
        ps = cs;
        pjx = cjx;
        pjy = cjy;
        pfl = cfl;
        pyr = yr;
    }
}

template <int S, bool TRT, bool SR, bool EXT = false>
__device__ __forceinline__ void step_tiles(const StepArgs &a, float *ring) {
    uint32_t mix = 0u;
    if constexpr (SR) mix = sr_step_mix(a.rng, a.par);
    const int tile = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= a.ntiles) return;   // uniform for the workgroup, before any barrier
    const int strip = tile / a.chunks, chunk = tile - strip * a.chunks;
    const int y0 = (int)(((int64_t)chunk * a.g.ny) / a.chunks);
    const int y1 = (int)(((int64_t)(chunk + 1) * a.g.ny) / a.chunks);
    step_tile<S, TRT, SR, EXT>(a.src, a.dst, a.flags, a.rowplain, a.g, a.m, strip * (int)blockDim.x, y0, y1,
                               (chunk & 1) == 0, ring, mix, a.acc);
}

// TRT selects the collision operator and SR the rounding of 16-bit stores at
// compile time (run-time branches would cost the paper's operator registers
// and occupancy).
template <int S, bool TRT, bool SR>
__global__ void __launch_bounds__(512) k_step(const StepArgs a) {
    extern __shared__ float ring[];
    step_tiles<S, TRT, SR>(a, ring);
}

// The fused kernel with a per-node acceleration field (StepArgs::acc), the
// paper's collision operator and nearest rounding.
template <int S>
__global__ void __launch_bounds__(512) k_step_acc(const StepArgs a) {
    extern __shared__ float ring[];
    step_tiles<S, false, false, true>(a, ring);
}

// The same kernel compiled for 8 resident waves per SIMD (64 VGPRs) instead of
// the 7 its natural register count allows.  The compiler keeps a few
// loop-invariant values in scratch (12 bytes per lane, reloaded per row from
// the L1 cache) and schedules the row loop differently.  Same arithmetic,
// bitwise the same results; which one is faster depends on the storage width
// and tile (the autotuner decides).
template <int S, bool TRT, bool SR>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(8, 8))) k_step8(const StepArgs a) {
    extern __shared__ float ring[];
    step_tiles<S, TRT, SR>(a, ring);
}

// ---------------------------------------------------------------------------
// K time steps per launch (temporal blocking, K = 2 or 3).  A step moves every
// population through HBM once each way; K steps in one pass move them once
// for all K, with the intermediate post-collision rows kept in LDS in the
// storage format, so the result is bitwise that of K single steps (each level
// decodes exactly what the level below would have stored).
//
// Each level of the dependency chain uses up one column and one row on each
// side twice (its pull reads the neighbours of the level below; its collision
// needs the neighbours' phi), so with H = 2K - 1 a workgroup of BX threads
// covers BX - 2H output columns (thread t works on column x0 - H + t,
// periodic) and a chunk of rows [y0, y1) marches through rows y0 - H .. y1 +
// H - 1.  Iteration i of the march (row a_i), for levels k = 0 .. K-1:
//   A:    pull row a_i from HBM (prefetched one row ahead), rho and phi of
//         level 0, phi and the flag word into LDS rings;             barrier
//   B_0:  level-0 collision of row a_{i-1} (phi of rows a_{i-2..i}), its
//         nine results, encoded, into the LDS ring F_0;               barrier
//   C_k:  (k >= 1) level-k pull of row a_{i-2k} from F_{k-1} (rows
//         a_{i-2k-1..i-2k+1}, bounce-back from the node's own results), rho
//         and phi of level k;                                         barrier
//   B_k:  level-k collision of row a_{i-2k-1} (phi rows a_{i-2k-2..i-2k}),
//         into F_k, or for the last level stored to HBM;  barrier (not last)
// B_k uses the pulled values C_k produced one iteration earlier (carried in
// registers).  The phi and F rings hold three rows (slot of row a_j: j mod 3)
// and the flag ring four (K = 2) or eight rows (slot j mod FR); every slot is
// rewritten only after a barrier that follows its last read.  Threads outside
// [H, H + nact) and rows outside the chunk are computed for their neighbours
// and not stored.
template <int K> struct Multi {
    static constexpr int H = 2 * K - 1;       // halo columns and rows per side
    static constexpr int FR = K == 2 ? 4 : 8; // flag ring rows (holds row a_{i-2(K-1)} while a_i is written)
};

template <int S, int K>
constexpr size_t multi_lds_bytes(int bx) {
    return (size_t)K * 3 * (bx + 2) * sizeof(float) + (size_t)Multi<K>::FR * bx * sizeof(uint16_t) +
           (size_t)(K - 1) * 3 * 9 * (bx + 2) * sizeof(typename Codec<S>::T);
}

// Slot of row a_{i-d} in a three-row ring, from the slot s0 of row a_i.
template <int D>
__device__ __forceinline__ int slot_back(int s0) {
    constexpr int r = D % 3;
    if constexpr (r == 0) return s0;
    else return s0 >= r ? s0 - r : s0 + 3 - r;
}

template <int S, bool TRT, bool SR, int BX, int K>
__device__ __forceinline__ void stepk_tile(const StepArgs &a, int x0, int y0, int y1, bool up, char *lds,
                                           const uint32_t (&mix)[K]) {
    using C = Codec<S>;
    using T = typename C::T;
    constexpr uint32_t E = sizeof(T);
    constexpr int H = Multi<K>::H, FR = Multi<K>::FR;
    const Grid &g = a.g;
    const Model &m = a.m;
    constexpr int P = BX + 2;   // ring rows carry one padding slot per side (compile-time strides)
    const int tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny;
    const uint32_t pitch = (uint32_t)g.pitch, plane = g.plane;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.src, 9u * plane * E);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(a.dst, 9u * plane * E);
    const __amdgpu_buffer_rsrc_t rf = make_rsrc(a.flags, plane * 2u);
    const int nrows = y1 - y0 + 2 * H;

    const int nact = min(BX - 2 * H, nx - x0);
    const bool out_col = tid >= H && tid < H + nact;
    int xc = (x0 - H + tid) % nx;
    if (xc < 0) xc += nx;
    const uint32_t x = (uint32_t)xc;
    const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == (uint32_t)nx - 1 ? 0 : x + 1;

    float *psi = reinterpret_cast<float *>(lds);                     // phi of level k  [K][3][P]
    uint16_t *flr = reinterpret_cast<uint16_t *>(psi + K * 3 * P);   // flag words      [FR][BX]
    T *F = reinterpret_cast<T *>(flr + FR * BX);                     // level-k results [K-1][3][9][P]
    if (tid < 6) {      // padding slots (read only by threads whose results are unused)
        const int r = tid >> 1, side = (tid & 1) ? P - 1 : 0;
#pragma unroll
        for (int k = 0; k < K; ++k) psi[(k * 3 + r) * P + side] = 0.f;
#pragma unroll
        for (int k = 0; k < K - 1; ++k)
#pragma unroll
            for (int q = 0; q < 9; ++q) F[((k * 3 + r) * 9 + q) * P + side] = C::enc(0.f);
    }

    auto row_at = [&](int i) { return wrapi(up ? y0 - H + i : y1 + H - 1 - i, ny); };

    const uint32_t v0 = x * E, vm = xm * E, vp = xp * E, vf = x * 2u;
    T raw[9];
    auto issue_pops = [&](int yr, uint32_t fl) {
        const int ym = yr == 0 ? ny - 1 : yr - 1, yp = yr == ny - 1 ? 0 : yr + 1;
        const uint32_t r0 = (uint32_t)yr * pitch, rm = (uint32_t)ym * pitch, rp = (uint32_t)yp * pitch;
        if (__builtin_amdgcn_ballot_w64((fl & 0xFFu) != 0u) == 0) {
            raw[0] = bload<T>(rs, v0, (0u * plane + r0) * E);
            raw[1] = bload<T>(rs, vm, (1u * plane + r0) * E);
            raw[2] = bload<T>(rs, v0, (2u * plane + rm) * E);
            raw[3] = bload<T>(rs, vp, (3u * plane + r0) * E);
            raw[4] = bload<T>(rs, v0, (4u * plane + rp) * E);
            raw[5] = bload<T>(rs, vm, (5u * plane + rm) * E);
            raw[6] = bload<T>(rs, vp, (6u * plane + rm) * E);
            raw[7] = bload<T>(rs, vp, (7u * plane + rp) * E);
            raw[8] = bload<T>(rs, vm, (8u * plane + rp) * E);
        } else {
            uint32_t o[9];
            pull_offsets(fl & 0xFFu, plane, rm, r0, rp, xm, x, xp, o);
#pragma unroll
            for (int q = 0; q < 9; ++q) raw[q] = bload<T>(rs, o[q] * E, 0u);
        }
    };
    auto load_flags = [&](int yr) { return bload_flag(rf, vf, (uint32_t)yr * pitch * 2u); };

    // per level: pulled populations (decoded), moments, flag word and row of
    // the row its next collision takes
    float pd[K][9], ps[K], pjx[K], pjy[K];
    uint32_t pfl[K];
    int pyr[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
#pragma unroll
        for (int q = 0; q < 9; ++q) pd[k][q] = 0.f;
        ps[k] = pjx[k] = pjy[k] = 0.f;
        pfl[k] = FL_SOLID;
        pyr[k] = 0;
    }

    // collision of level k from its carried values; results encoded (nearest or
    // stochastic with the level's mix) into out
    auto collide_level = [&](auto kc, const float *rowm, const float *row0, const float *rowp, T out[9]) {
        constexpr int k = decltype(kc)::value;
        float p[9];
        collide_post<TRT>(m, pd[k], ps[k], pjx[k], pjy[k], pfl[k], rowm, row0, rowp, tid + 1, p);
        if constexpr (SR) {
            const uint32_t k0 = ((uint32_t)pyr[k] * pitch + x) * 5u;
            uint32_t h[5];
#pragma unroll
            for (int j = 0; j < 5; ++j) h[j] = lowbias32((k0 + (uint32_t)j) ^ mix[k]);
#pragma unroll
            for (int q = 0; q < 9; ++q) out[q] = C::enc_sr(p[q], (q & 1) ? (h[q >> 1] >> 16) : (h[q >> 1] & 0xFFFFu));
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q) out[q] = C::enc(p[q]);
        }
    };
    // level k >= 1 pull of row a_{i-2k} (slot k0 of ring F_{k-1}; km / kp: rows y -+ 1)
    auto pull_level = [&](const T *Fb, int ks, int km, int kp, uint32_t nb, float d[9]) {
        const T *Fk = Fb + ks * 9 * P + tid + 1, *Fm = Fb + km * 9 * P + tid + 1, *Fp = Fb + kp * 9 * P + tid + 1;
        // population a from x - e_a, or (bounce-back) opp(a) of the node itself;
        // a wave none of whose nodes has a solid neighbour skips the selection
        T v[9];
        v[0] = Fk[0 * P];
        if (__builtin_amdgcn_ballot_w64(nb != 0u) == 0) {
            v[1] = Fk[1 * P - 1];
            v[2] = Fm[2 * P];
            v[3] = Fk[3 * P + 1];
            v[4] = Fp[4 * P];
            v[5] = Fm[5 * P - 1];
            v[6] = Fm[6 * P + 1];
            v[7] = Fp[7 * P + 1];
            v[8] = Fp[8 * P - 1];
        } else {
            v[1] = (nb & 0x04u) ? Fk[3 * P] : Fk[1 * P - 1];
            v[2] = (nb & 0x08u) ? Fk[4 * P] : Fm[2 * P];
            v[3] = (nb & 0x01u) ? Fk[1 * P] : Fk[3 * P + 1];
            v[4] = (nb & 0x02u) ? Fk[2 * P] : Fp[4 * P];
            v[5] = (nb & 0x40u) ? Fk[7 * P] : Fm[5 * P - 1];
            v[6] = (nb & 0x80u) ? Fk[8 * P] : Fm[6 * P + 1];
            v[7] = (nb & 0x10u) ? Fk[5 * P] : Fp[7 * P + 1];
            v[8] = (nb & 0x20u) ? Fk[6 * P] : Fp[8 * P - 1];
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) d[q] = C::dec(v[q]);
    };

    uint32_t fl1, fl2;
    {
        const uint32_t f0 = load_flags(row_at(0));
        fl2 = load_flags(row_at(1));
        issue_pops(row_at(0), f0);
        fl1 = f0;
    }

    int s0 = 0;     // slot of row a_i in the three-row rings (i mod 3)
    for (int i = 0; i < nrows; ++i, s0 = s0 == 2 ? 0 : s0 + 1) {
        // A: row a_i, level 0
        const int yr = row_at(i);
        const uint32_t cfl = fl1;
        T craw[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) craw[q] = raw[q];
        fl1 = fl2;
        fl2 = load_flags(row_at(min(i + 2, nrows - 1)));
        issue_pops(row_at(min(i + 1, nrows - 1)), fl1);
        float cd[9], cs, cjx, cjy;
#pragma unroll
        for (int q = 0; q < 9; ++q) cd[q] = C::dec(craw[q]);
        moments9(cd, cs, cjx, cjy);
        psi[s0 * P + tid + 1] = (cfl & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + cs);
        flr[(i & (FR - 1)) * BX + tid] = (uint16_t)cfl;
        lds_barrier();

        // B_0: level-0 collision of row a_{i-1} into F_0 (or, for K = 1, HBM)
        {
            const float *older = psi + slot_back<2>(s0) * P, *mid = psi + slot_back<1>(s0) * P,
                        *newer = psi + s0 * P;
            if (i >= 2 && !(pfl[0] & FL_SOLID)) {
                T o[9];
                collide_level(std::integral_constant<int, 0>{}, up ? older : newer, mid, up ? newer : older, o);
                T *fr = F + slot_back<1>(s0) * 9 * P + tid + 1;
#pragma unroll
                for (int q = 0; q < 9; ++q) fr[q * P] = o[q];
            }
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) pd[0][q] = cd[q];
        ps[0] = cs;
        pjx[0] = cjx;
        pjy[0] = cjy;
        pfl[0] = cfl;
        pyr[0] = yr;
        lds_barrier();

        // levels 1 .. K-1: C_k, barrier, B_k (barrier between levels)
        auto level = [&](auto kc) {
            constexpr int k = decltype(kc)::value;
            // C_k: pull of row a_{i-2k} from F_{k-1}, rho and phi of level k
            float ed[9], es = 0.f, ejx = 0.f, ejy = 0.f;
            uint32_t efl = FL_SOLID;
            const int sk = slot_back<2 * k>(s0);
            if (i >= 4 * k) {
                const int km = up ? slot_back<2 * k + 1>(s0) : slot_back<2 * k - 1>(s0);   // row y - 1
                const int kp = up ? slot_back<2 * k - 1>(s0) : slot_back<2 * k + 1>(s0);   // row y + 1
                efl = flr[((i - 2 * k) & (FR - 1)) * BX + tid];
                pull_level(F + (k - 1) * 3 * 9 * P, sk, km, kp, efl & 0xFFu, ed);
                moments9(ed, es, ejx, ejy);
                psi[(k * 3 + sk) * P + tid + 1] = (efl & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + es);
            } else {
#pragma unroll
                for (int q = 0; q < 9; ++q) ed[q] = 0.f;
            }
            lds_barrier();
            // B_k: level-k collision of row a_{i-2k-1} (phi rows a_{i-2k-2 .. i-2k})
            const float *pk = psi + k * 3 * P;
            const float *older = pk + slot_back<2 * k + 2>(s0) * P, *mid = pk + slot_back<2 * k + 1>(s0) * P,
                        *newer = pk + sk * P;
            if constexpr (k == K - 1) {
                if (i >= 4 * k + 2 && out_col && !(pfl[k] & FL_SOLID)) {
                    T o[9];
                    collide_level(kc, up ? older : newer, mid, up ? newer : older, o);
                    const uint32_t prow = (uint32_t)pyr[k] * pitch;
#pragma unroll
                    for (int q = 0; q < 9; ++q) bstore(rd, v0, ((uint32_t)q * plane + prow) * E, o[q]);
                }
            } else {
                if (i >= 4 * k + 2 && !(pfl[k] & FL_SOLID)) {
                    T o[9];
                    collide_level(kc, up ? older : newer, mid, up ? newer : older, o);
                    T *fr = F + (k * 3 + slot_back<2 * k + 1>(s0)) * 9 * P + tid + 1;
#pragma unroll
                    for (int q = 0; q < 9; ++q) fr[q * P] = o[q];
                }
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) pd[k][q] = ed[q];
            ps[k] = es;
            pjx[k] = ejx;
            pjy[k] = ejy;
            pfl[k] = efl;
            pyr[k] = row_at(i - 2 * k >= 0 ? i - 2 * k : 0);
            if constexpr (k < K - 1) lds_barrier();
        };
        level(std::integral_constant<int, 1>{});
        if constexpr (K >= 3) level(std::integral_constant<int, 2>{});
    }
}

template <int S, bool TRT, bool SR, int BX, int K>
__global__ void __launch_bounds__(BX) k_stepk(const StepArgs a) {
    extern __shared__ char ldsk[];
    uint32_t mix[K];
#pragma unroll
    for (int k = 0; k < K; ++k) mix[k] = 0u;
    if constexpr (SR) {
        // the step counts of the K steps; the next launch reads count + K
        const uint32_t count = a.rng[a.par];
        if (blockIdx.x == 0 && threadIdx.x == 0) a.rng[a.par ^ 1] = count + (uint32_t)K;
#pragma unroll
        for (int k = 0; k < K; ++k) mix[k] = lowbias32(count + (uint32_t)k + 0x9e3779b9u);
    }
    const int tile = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= a.ntiles) return;   // uniform for the workgroup, before any barrier
    const int strip = tile / a.chunks, chunk = tile - strip * a.chunks;
    const int y0 = (int)(((int64_t)chunk * a.g.ny) / a.chunks);
    const int y1 = (int)(((int64_t)(chunk + 1) * a.g.ny) / a.chunks);
    stepk_tile<S, TRT, SR, BX, K>(a, strip * (BX - 2 * Multi<K>::H), y0, y1, (chunk & 1) == 0, ldsk, mix);
}

// ---------------------------------------------------------------------------
// Wide step: step_tile with V adjacent columns per thread, so that a row of
// one population plane moves as V * sizeof(T) bytes per lane (8 or 16 bytes
// instead of 4 or 2), which the memory pipeline streams markedly faster.  Per
// node the arithmetic is that of step_tile (bitwise the same results).  A
// wave whose columns do not wrap and none of whose nodes in the row has a
// solid neighbour pulls each plane as one V-wide load from column x - e_a
// (4-byte aligned for FP32, 2-byte for 16-bit data); otherwise each node
// pulls its nine populations one by one.  A thread whose V nodes are all
// active fluid nodes stores each plane as one V-wide store.
template <int N> struct UWord;
template <> struct UWord<4> { using U = uint32_t; };
template <> struct UWord<8> { using U = __attribute__((ext_vector_type(2))) uint32_t; };
template <> struct UWord<16> { using U = __attribute__((ext_vector_type(4))) uint32_t; };

template <class T, int V>
__device__ __forceinline__ void bload_vec(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, T out[V]) {
    constexpr int N = V * (int)sizeof(T);
    using U = typename UWord<N>::U;
    U w;
    if constexpr (N == 4) w = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
    else if constexpr (N == 8) w = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    else w = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
    struct Pack { T v[V]; };
    const Pack pk = __builtin_bit_cast(Pack, w);
#pragma unroll
    for (int j = 0; j < V; ++j) out[j] = pk.v[j];
}

template <class T, int V>
__device__ __forceinline__ void bstore_vec(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, const T in[V]) {
    constexpr int N = V * (int)sizeof(T);
    using U = typename UWord<N>::U;
    struct Pack { T v[V]; };
    Pack pk;
#pragma unroll
    for (int j = 0; j < V; ++j) pk.v[j] = in[j];
    const U w = __builtin_bit_cast(U, pk);
    if constexpr (N == 4) __builtin_amdgcn_raw_buffer_store_b32(w, r, (int)voff, (int)soff, kStoreNT);
    else if constexpr (N == 8) __builtin_amdgcn_raw_buffer_store_b64(w, r, (int)voff, (int)soff, kStoreNT);
    else __builtin_amdgcn_raw_buffer_store_b128(w, r, (int)voff, (int)soff, kStoreNT);
}

template <int S, int V>
__device__ __forceinline__ void step_tile_wide(const void *src_ptr, void *dst_ptr, const uint16_t *flags_ptr,
                                               const Grid &g, const Model &m, int x0, int y0, int y1, bool up,
                                               float *ring) {
    using C = Codec<S>;
    using T = typename C::T;
    const int BX = blockDim.x;
    const int NC = BX * V, W = NC + 2;      // columns of the strip, LDS ring row width
    const int tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny;
    const uint32_t pitch = (uint32_t)g.pitch, plane = g.plane;
    constexpr uint32_t E = sizeof(T);
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src_ptr, 9u * plane * E);
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(dst_ptr, 9u * plane * E);
    const __amdgpu_buffer_rsrc_t rf = make_rsrc(flags_ptr, plane * 2u);
    const int nrows = y1 - y0 + 2;

    const int nact = min(NC, nx - x0);
    const int c0 = V * tid;                   // first column of this thread in the strip
    bool act[V];
    uint32_t xj[V], xmj[V], xpj[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
        act[j] = c0 + j < nact;
        const int x = x0 + (act[j] ? c0 + j : 0);
        xj[j] = (uint32_t)x;
        xmj[j] = x == 0 ? nx - 1 : x - 1;
        xpj[j] = x == nx - 1 ? 0 : x + 1;
    }
    bool all_act = true;
#pragma unroll
    for (int j = 0; j < V; ++j) all_act = all_act && act[j];

    // halo gather lanes: 0..8 left column, 16..24 right column, one population each
    const int hl = tid & 15;
    const bool hlane = tid < 32 && hl < 9;
    const int hx = (tid < 16) ? (x0 == 0 ? nx - 1 : x0 - 1) : (x0 + nact == nx ? 0 : x0 + nact);
    const int ha = hlane ? hl : 0;
    const uint32_t hsx = (uint32_t)wrapi(hx - kEX[ha], nx);
    const int hdy = -kEY[ha];
    const uint32_t hsrcbit = kSRCBIT[ha];
    const uint32_t hopp = (uint32_t)kOPP[ha];

    auto row_at = [&](int i) {
        const int r = up ? y0 - 1 + i : y1 - i;
        return wrapi(r, ny);
    };

    uint32_t fl1[V], fl2[V];
    uint32_t hfl1 = FL_SOLID, hfl2 = FL_SOLID;
#pragma unroll
    for (int j = 0; j < V; ++j) fl1[j] = fl2[j] = FL_SOLID;
    T raw[9][V];
    T hraw = C::enc(0.f);
    float pd[9][V], ps[V], pjx[V], pjy[V];
    uint32_t pfl[V];
#pragma unroll
    for (int j = 0; j < V; ++j) {
#pragma unroll
        for (int q = 0; q < 9; ++q) pd[q][j] = 0.f;
        ps[j] = pjx[j] = pjy[j] = 0.f;
        pfl[j] = FL_SOLID;
    }
    int pyr = 0;

    // the wave's columns and their x-neighbours do not wrap, and all are active
    const int wave_c0 = V * (tid & ~63);
    const bool wave_inner = x0 + wave_c0 >= 1 && x0 + wave_c0 + 64 * V <= nx - 1 && wave_c0 + 64 * V <= nact;
    const uint32_t vbase = (uint32_t)(x0 + c0);
    auto issue_pops = [&](int yr, const uint32_t (&fl)[V], uint32_t hfl) {
        const int ym = yr == 0 ? ny - 1 : yr - 1, yp = yr == ny - 1 ? 0 : yr + 1;
        const uint32_t r0 = (uint32_t)yr * pitch, rm = (uint32_t)ym * pitch, rp = (uint32_t)yp * pitch;
        uint32_t walls = 0u;
#pragma unroll
        for (int j = 0; j < V; ++j) walls |= fl[j] & 0xFFu;
        if (wave_inner && __builtin_amdgcn_ballot_w64(walls != 0u) == 0) {
            // population a of column x comes from column x - e_a of row y - e_a
            bload_vec<T, V>(rs, vbase * E, (0u * plane + r0) * E, raw[0]);
            bload_vec<T, V>(rs, (vbase - 1u) * E, (1u * plane + r0) * E, raw[1]);
            bload_vec<T, V>(rs, vbase * E, (2u * plane + rm) * E, raw[2]);
            bload_vec<T, V>(rs, (vbase + 1u) * E, (3u * plane + r0) * E, raw[3]);
            bload_vec<T, V>(rs, vbase * E, (4u * plane + rp) * E, raw[4]);
            bload_vec<T, V>(rs, (vbase - 1u) * E, (5u * plane + rm) * E, raw[5]);
            bload_vec<T, V>(rs, (vbase + 1u) * E, (6u * plane + rm) * E, raw[6]);
            bload_vec<T, V>(rs, (vbase + 1u) * E, (7u * plane + rp) * E, raw[7]);
            bload_vec<T, V>(rs, (vbase - 1u) * E, (8u * plane + rp) * E, raw[8]);
        } else {
#pragma unroll
            for (int j = 0; j < V; ++j) {
                uint32_t o[9];
                pull_offsets(fl[j] & 0xFFu, plane, rm, r0, rp, xmj[j], xj[j], xpj[j], o);
#pragma unroll
                for (int q = 0; q < 9; ++q) raw[q][j] = bload<T>(rs, o[q] * E, 0u);
            }
        }
        if (tid < 64) {
            const uint32_t hrow = hdy < 0 ? rm : (hdy > 0 ? rp : r0);
            const uint32_t off = (hfl & hsrcbit) ? hopp * plane + r0 + (uint32_t)hx
                                                 : (uint32_t)ha * plane + hrow + hsx;
            hraw = bload<T>(rs, off * E, 0u);
        }
    };
    const uint32_t vhf = (uint32_t)hx * 2u;
    auto issue_flags = [&](int yr, uint32_t (&fl)[V], uint32_t &hfl) {
        const uint32_t r0b = (uint32_t)yr * pitch * 2u;
#pragma unroll
        for (int j = 0; j < V; ++j) fl[j] = bload_flag(rf, xj[j] * 2u, r0b);
        if (tid < 64) hfl = bload_flag(rf, vhf, r0b);
    };

    // prologue: flags of rows 0 and 1, populations of row 0
    issue_flags(row_at(0), fl1, hfl1);
    issue_flags(row_at(1), fl2, hfl2);
    issue_pops(row_at(0), fl1, hfl1);

    for (int i = 0; i < nrows; ++i) {
        const int yr = row_at(i);
        // row i from the pipeline, decoded; then rows i+1 (populations) and i+2 (flags)
        uint32_t cfl[V];
        float cd[9][V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            cfl[j] = fl1[j];
#pragma unroll
            for (int q = 0; q < 9; ++q) cd[q][j] = C::dec(raw[q][j]);
        }
        const uint32_t chfl = hfl1;
        const float hv = (hlane && !(chfl & FL_SOLID)) ? C::dec(hraw) : 0.f;
#pragma unroll
        for (int j = 0; j < V; ++j) fl1[j] = fl2[j];
        hfl1 = hfl2;
        issue_flags(row_at(min(i + 2, nrows - 1)), fl2, hfl2);
        issue_pops(row_at(min(i + 1, nrows - 1)), fl1, hfl1);

        float *slot = ring + (i & (RING - 1)) * W;
        float cs[V], cjx[V], cjy[V];
#pragma unroll
        for (int j = 0; j < V; ++j) {
            float d[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) d[q] = cd[q][j];
            moments9(d, cs[j], cjx[j], cjy[j]);
            if (act[j]) slot[c0 + j + 1] = (cfl[j] & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + cs[j]);
        }
        if (tid < 64) {
            const int base = tid & ~15;
            float gq[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) gq[q] = __shfl(hv, base + q, 64);
            if (tid == 0 || tid == 16) {
                const float hs = (((gq[0] + gq[1]) + (gq[2] + gq[3])) + ((gq[4] + gq[5]) + (gq[6] + gq[7]))) + gq[8];
                const float phi = (chfl & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + hs);
                slot[tid == 0 ? 0 : nact + 1] = phi;
            }
        }
        lds_barrier();
        if (i >= 2) {
            const float *older = ring + ((i - 2) & (RING - 1)) * W;
            const float *mid = ring + ((i - 1) & (RING - 1)) * W;
            const float *rowm = up ? older : slot;
            const float *rowp = up ? slot : older;
            const uint32_t prow = (uint32_t)pyr * pitch;
            T out[V][9];
            bool fluid_all = all_act;
#pragma unroll
            for (int j = 0; j < V; ++j) {
                fluid_all = fluid_all && !(pfl[j] & FL_SOLID);
                if (act[j] && !(pfl[j] & FL_SOLID)) {
                    float d[9];
#pragma unroll
                    for (int q = 0; q < 9; ++q) d[q] = pd[q][j];
                    collide<C>(m, d, ps[j], pjx[j], pjy[j], pfl[j], rowm, mid, rowp, c0 + j + 1, out[j]);
                }
            }
            if (fluid_all) {
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    T v[V];
#pragma unroll
                    for (int j = 0; j < V; ++j) v[j] = out[j][q];
                    bstore_vec<T, V>(rd, vbase * E, ((uint32_t)q * plane + prow) * E, v);
                }
            } else {
#pragma unroll
                for (int j = 0; j < V; ++j)
                    if (act[j] && !(pfl[j] & FL_SOLID)) {
#pragma unroll
                        for (int q = 0; q < 9; ++q)
                            bstore(rd, xj[j] * E, ((uint32_t)q * plane + prow) * E, out[j][q]);
                    }
            }
        }
#pragma unroll
        for (int j = 0; j < V; ++j) {
#pragma unroll
            for (int q = 0; q < 9; ++q) pd[q][j] = cd[q][j];
            ps[j] = cs[j];
            pjx[j] = cjx[j];
            pjy[j] = cjy[j];
            pfl[j] = cfl[j];
        }
        pyr = yr;
    }
}

template <int S, int V>
__global__ void __launch_bounds__(512) k_step_wide(const StepArgs a) {
    extern __shared__ float ring[];
    const int tile = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= a.ntiles) return;   // uniform for the workgroup, before any barrier
    const int strip = tile / a.chunks, chunk = tile - strip * a.chunks;
    const int y0 = (int)(((int64_t)chunk * a.g.ny) / a.chunks);
    const int y1 = (int)(((int64_t)(chunk + 1) * a.g.ny) / a.chunks);
    step_tile_wide<S, V>(a.src, a.dst, a.flags, a.g, a.m, strip * (int)blockDim.x * V, y0, y1,
                         (chunk & 1) == 0, ring);
}

// ---------------------------------------------------------------------------
// Split step: the arithmetic of step_tile, bitwise, with the HBM reads moved
// to a producer wave.
//
// A wave that both loads and stores cannot keep loads in flight across its
// own waits: its stores and loads share one counter, so waiting for a load
// also waits for every store before it.  Here the BX compute threads (the
// consumer waves) only read LDS and store, and one producer wave only loads:
// it streams each pulled row straight into an LDS ring with direct-to-LDS
// buffer loads, two rows ahead of the consumers, and its waits count loads
// only.  Per row the producer resolves the bounce-back addresses from the flag
// words (loaded two rows ahead into registers) and also copies the flag words
// into LDS for the consumers.  One workgroup barrier per row, as in step_tile.
//
// LDS: NR = 3 row slots of 9 x BX populations plus 18 halo populations (one
// dword per value; 16-bit values arrive zero-extended in the low half; slots
// 16-byte aligned for the 16-byte loads), 3 slots
// of BX + 2 flag words, and the 4-row phi ring.
constexpr int SPLIT_NR = 3;

template <int S>
__device__ __forceinline__ float dec_word(uint32_t w) {
    using C = Codec<S>;
    using T = typename C::T;
    if constexpr (sizeof(T) == 4) return C::dec(__builtin_bit_cast(T, w));
    else return C::dec(__builtin_bit_cast(T, (unsigned short)(w & 0xFFFFu)));
}

// Direct-to-LDS load: lane l writes lds[l] (one dword) with BYTES bytes read
// at byte offset voff of the buffer.
template <int BYTES>
__device__ __forceinline__ void dma(__amdgpu_buffer_rsrc_t r, uint32_t *lds, uint32_t voff) {
    static_assert(BYTES == 2 || BYTES == 4, "2- or 4-byte loads");
    auto *p = (__attribute__((address_space(3))) void *)lds;
    if constexpr (BYTES == 4) __builtin_amdgcn_raw_ptr_buffer_load_lds(r, p, 4, (int)voff, 0, 0, 0);
    else __builtin_amdgcn_raw_ptr_buffer_load_lds(r, p, 2, (int)voff, 0, 0, 0);
}

// Wait until at most N vector-memory operations of this wave are outstanding
// (gfx9 encoding: vmcnt in bits 3:0 and 15:14; expcnt and lgkmcnt not waited).
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | ((N >> 4) << 14));
}

template <int S, int BX>
__global__ void __launch_bounds__(BX + 64) k_step_split(const StepArgs a) {
    using C = Codec<S>;
    constexpr uint32_t E = sizeof(typename C::T);
    constexpr int NG = BX / 64;                 // column groups of a producer lane
    constexpr int NF = NG + 1;                  // flag loads per row (own columns + halo)
    constexpr int NP = 9 * NG + 1 + NG + 1;     // LDS loads per row (populations + flags)
    constexpr int POPS = 9 * BX + 20;           // 18 halo values, rounded up to 16-byte slots
    __shared__ __attribute__((aligned(16))) uint32_t pring[SPLIT_NR][POPS];
    __shared__ uint32_t fring[SPLIT_NR][BX + 2];
    __shared__ float psi[RING][BX + 2];

    const int tile = (int)(blockIdx.x & 7u) * a.tiles_per_xcd + (int)(blockIdx.x >> 3);
    if (tile >= a.ntiles) return;   // uniform for the workgroup, before any barrier
    const int strip = tile / a.chunks, chunk = tile - strip * a.chunks;
    const int y0 = (int)(((int64_t)chunk * a.g.ny) / a.chunks);
    const int y1 = (int)(((int64_t)(chunk + 1) * a.g.ny) / a.chunks);
    const bool up = (chunk & 1) == 0;
    const Grid &g = a.g;
    const Model &m = a.m;
    const int nx = g.nx, ny = g.ny;
    const uint32_t pitch = (uint32_t)g.pitch, plane = g.plane;
    const int x0 = strip * BX;
    const int nrows = y1 - y0 + 2;       // the chunk plus one halo row per side
    const int nact = min(BX, nx - x0);
    const int tid = threadIdx.x;
    const int hxl = x0 == 0 ? nx - 1 : x0 - 1;
    const int hxr = x0 + nact == nx ? 0 : x0 + nact;
    auto row_at = [&](int i) {
        const int r = up ? y0 - 1 + i : y1 - i;
        return wrapi(r, ny);
    };

    if (tid >= BX) {
        // ---- producer wave
        const int lane = tid - BX;
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.src, 9u * plane * E);
        const __amdgpu_buffer_rsrc_t rf = make_rsrc(a.flags, plane * 2u);
        uint32_t xc[NG], xmc[NG], xpc[NG];
#pragma unroll
        for (int k = 0; k < NG; ++k) {
            const int c = 64 * k + lane;
            const int x = x0 + (c < nact ? c : 0);
            xc[k] = (uint32_t)x;
            xmc[k] = x == 0 ? nx - 1 : x - 1;
            xpc[k] = x == nx - 1 ? 0 : x + 1;
        }
        // halo populations: lanes 0..8 the left column, 9..17 the right one
        const int side = lane >= 9 ? 1 : 0;
        const int ha = lane < 18 ? lane - 9 * side : 0;
        const int hx = side ? hxr : hxl;
        const uint32_t hsx = (uint32_t)wrapi(hx - kEX[ha], nx);
        const int hdy = -kEY[ha];
        const uint32_t hsrcbit = kSRCBIT[ha];
        const uint32_t hopp = (uint32_t)kOPP[ha];
        const uint32_t hflag_x = (uint32_t)(lane == 1 ? hxr : hxl);   // flag copies: lane 0 left, 1 right

        auto load_flags = [&](int yr, uint32_t (&f)[NF]) {
            const uint32_t rb = (uint32_t)yr * pitch * 2u;
#pragma unroll
            for (int k = 0; k < NG; ++k) f[k] = bload_flag(rf, xc[k] * 2u, rb);
            f[NG] = bload_flag(rf, (uint32_t)hx * 2u, rb);
        };
        auto issue_row = [&](int yr, int slot, const uint32_t (&f)[NF]) {
            const int ym = yr == 0 ? ny - 1 : yr - 1, yp = yr == ny - 1 ? 0 : yr + 1;
            const uint32_t r0 = (uint32_t)yr * pitch, rm = (uint32_t)ym * pitch, rp = (uint32_t)yp * pitch;
            uint32_t *pr = pring[slot];
#pragma unroll
            for (int k = 0; k < NG; ++k) {
                uint32_t o[9];
                pull_offsets(f[k] & 0xFFu, plane, rm, r0, rp, xmc[k], xc[k], xpc[k], o);
#pragma unroll
                for (int q = 0; q < 9; ++q) dma<E>(rs, pr + q * BX + 64 * k, o[q] * E);
            }
            if (lane < 18) {
                const uint32_t hrow = hdy < 0 ? rm : (hdy > 0 ? rp : r0);
                const uint32_t off = (f[NG] & hsrcbit) ? hopp * plane + r0 + (uint32_t)hx
                                                       : (uint32_t)ha * plane + hrow + hsx;
                dma<E>(rs, pr + 9 * BX, off * E);
            }
            uint32_t *fr = fring[slot];
#pragma unroll
            for (int k = 0; k < NG; ++k) dma<2>(rf, fr + 64 * k, (r0 + xc[k]) * 2u);
            if (lane < 2) dma<2>(rf, fr + BX, (r0 + hflag_x) * 2u);
        };

        // Rows are issued two ahead of the consumers: at iteration i the
        // producer issues row i + 2 into slot (i + 2) % 3 (the slot of row
        // i - 1, read before barrier i - 1), loads the flags of row i + 4, and
        // waits until row i + 1 has landed before barrier i.  Past the end of
        // the chunk the last row is issued again (cache hits), so every
        // iteration has the same number of loads and the waits are exact.
        // Even and odd rows keep their flags in separate registers.
        uint32_t fe[NF], fo[NF];
        load_flags(row_at(0), fe);
        load_flags(row_at(1), fo);
        issue_row(row_at(0), 0, fe);
        load_flags(row_at(min(2, nrows - 1)), fe);
        issue_row(row_at(1), 1, fo);
        load_flags(row_at(min(3, nrows - 1)), fo);
        wait_vm<2 * NF + NP>();               // row 0 has landed
        __builtin_amdgcn_s_barrier();
        for (int i = 0; i < nrows; i += 2) {
            issue_row(row_at(min(i + 2, nrows - 1)), (i + 2) % SPLIT_NR, fe);
            load_flags(row_at(min(i + 4, nrows - 1)), fe);
            wait_vm<2 * NF + NP>();           // row i + 1 has landed
            __builtin_amdgcn_s_barrier();
            if (i + 1 < nrows) {
                issue_row(row_at(min(i + 3, nrows - 1)), (i + 3) % SPLIT_NR, fo);
                load_flags(row_at(min(i + 5, nrows - 1)), fo);
                wait_vm<2 * NF + NP>();       // row i + 2 has landed
                __builtin_amdgcn_s_barrier();
            }
        }
        wait_vm<0>();   // no load into LDS may land after the workgroup ends
        return;
    }

    // ---- consumer waves: one column per thread
    const __amdgpu_buffer_rsrc_t rd = make_rsrc(a.dst, 9u * plane * E);
    const bool act = tid < nact;
    const uint32_t v0 = (uint32_t)(x0 + (act ? tid : 0)) * E;
    float pd[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float ps = 0.f, pjx = 0.f, pjy = 0.f;
    uint32_t pfl = FL_SOLID;
    int pyr = 0;
    lds_barrier();
    for (int i = 0; i < nrows; ++i) {
        const int yr = row_at(i);
        const int sl = i % SPLIT_NR;
        const uint32_t *pr = pring[sl];
        float cd[9], cs = 0.f, cjx = 0.f, cjy = 0.f;
#pragma unroll
        for (int q = 0; q < 9; ++q) cd[q] = dec_word<S>(pr[q * BX + tid]);
        const uint32_t cfl = fring[sl][tid] & 0xFFFFu;
        moments9(cd, cs, cjx, cjy);
        float *slot = psi[i & (RING - 1)];
        if (act) slot[tid + 1] = (cfl & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + cs);
        if (tid < 2) {
            // rho of a halo node from its nine populations, in the order of moments9
            float hd[9], hs = 0.f, hjx = 0.f, hjy = 0.f;
#pragma unroll
            for (int q = 0; q < 9; ++q) hd[q] = dec_word<S>(pr[9 * BX + 9 * tid + q]);
            const uint32_t hfl = fring[sl][BX + tid] & 0xFFFFu;
            moments9(hd, hs, hjx, hjy);
            slot[tid == 0 ? 0 : nact + 1] = (hfl & FL_SOLID) ? 0.f : pseudopotential(m, m.rho_off + hs);
        }
        lds_barrier();
        if (i >= 2 && act && !(pfl & FL_SOLID)) {
            const float *older = psi[(i - 2) & (RING - 1)];
            const float *mid = psi[(i - 1) & (RING - 1)];
            const float *rowm = up ? older : slot;
            const float *rowp = up ? slot : older;
            collide_store<C>(m, pd, ps, pjx, pjy, pfl, rowm, mid, rowp, tid + 1, rd, plane,
                             (uint32_t)pyr * pitch, v0);
        }
#pragma unroll
        for (int q = 0; q < 9; ++q) pd[q] = cd[q];
        ps = cs;
        pjx = cjx;
        pjy = cjy;
        pfl = cfl;
        pyr = yr;
    }
}

// Populations at t = 0: f_a = f_a^eq(rho, u) of eq. (3), written where the
// first pull will find them (the inverse of streaming with bounce-back).
template <int S>
__global__ void k_init(typename Codec<S>::T *__restrict__ dst, const uint16_t *__restrict__ flags,
                       Grid g, const float *__restrict__ rho_in,
                       const float *__restrict__ ux_in, const float *__restrict__ uy_in,
                       int dense_pitch, float rho_off) {
    using C = Codec<S>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nx) return;
    const uint32_t pitch = (uint32_t)g.pitch, plane = g.plane;
    const uint32_t own = (uint32_t)y * pitch + x;
    const uint32_t fl = flags[own];
    if (fl & FL_SOLID) return;
    const int di = y * dense_pitch + x;
    const float rho = rho_in[di], ux = ux_in ? ux_in[di] : 0.f, uy = uy_in ? uy_in[di] : 0.f;
    const uint32_t xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const uint32_t rm = (uint32_t)(y == 0 ? g.ny - 1 : y - 1) * pitch;
    const uint32_t r0 = (uint32_t)y * pitch;
    const uint32_t rp = (uint32_t)(y == g.ny - 1 ? 0 : y + 1) * pitch;
    float feq[9];
    equilibrium(rho, rho - rho_off, rho * ux, rho * uy, feq);
    // target of population a: node x - e_a in plane a, or plane opp(a) of x
    st(dst, own, C::enc(feq[0]));
    st(dst, (fl & 0x04u) ? 3u * plane + own : 1u * plane + r0 + xm, C::enc(feq[1]));
    st(dst, (fl & 0x08u) ? 4u * plane + own : 2u * plane + rm + x, C::enc(feq[2]));
    st(dst, (fl & 0x01u) ? 1u * plane + own : 3u * plane + r0 + xp, C::enc(feq[3]));
    st(dst, (fl & 0x02u) ? 2u * plane + own : 4u * plane + rp + x, C::enc(feq[4]));
    st(dst, (fl & 0x40u) ? 7u * plane + own : 5u * plane + rm + xm, C::enc(feq[5]));
    st(dst, (fl & 0x80u) ? 8u * plane + own : 6u * plane + rm + xp, C::enc(feq[6]));
    st(dst, (fl & 0x10u) ? 5u * plane + own : 7u * plane + rp + xp, C::enc(feq[7]));
    st(dst, (fl & 0x20u) ? 6u * plane + own : 8u * plane + rp + xm, C::enc(feq[8]));
}

__global__ void k_fill(uint4 *__restrict__ p, size_t n16) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n16; i += stride) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Streaming copy: the practical HBM ceiling the step kernels are measured
// against (a copy moves the bytes a step moves, with no stencil).  One pass:
// lane i of the grid copies the U 16-byte chunks i, i + T, ..., i + (U-1) T of
// its workgroup's range (T threads per workgroup) with non-temporal loads and
// stores, all loads before the stores, and the workgroup exits.  Short-lived
// workgroups keep the concurrently touched memory in a narrow band, which the
// memory system streams faster than long-running loops over the whole buffer.
using v4u = __attribute__((ext_vector_type(4))) uint32_t;
template <int U>
__global__ void __launch_bounds__(256) k_stream_copy(v4u *__restrict__ dst, const v4u *__restrict__ src,
                                                     size_t n16) {
    const size_t base = (size_t)blockIdx.x * blockDim.x * U + threadIdx.x;
    v4u v[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const size_t i = base + (size_t)k * blockDim.x;
        if (i < n16) v[k] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
        const size_t i = base + (size_t)k * blockDim.x;
        if (i < n16) __builtin_nontemporal_store(v[k], dst + i);
    }
}

// eq. (2) moments of the current state into dense float32 [ny][nx] arrays.
template <int S>
__global__ void k_moments(const typename Codec<S>::T *__restrict__ src,
                          const uint16_t *__restrict__ flags, Grid g, float rho_off,
                          float *__restrict__ rho_out, float *__restrict__ ux_out,
                          float *__restrict__ uy_out) {
    using C = Codec<S>;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= g.nx) return;
    const uint32_t pitch = (uint32_t)g.pitch;
    const uint32_t r0 = (uint32_t)y * pitch;
    const uint32_t fl = flags[r0 + x];
    float rho = 0.f, ux = 0.f, uy = 0.f;
    if (!(fl & FL_SOLID)) {
        const uint32_t xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
        const uint32_t rm = (uint32_t)(y == 0 ? g.ny - 1 : y - 1) * pitch;
        const uint32_t rp = (uint32_t)(y == g.ny - 1 ? 0 : y + 1) * pitch;
        float d[9], sd, jx, jy;
        pull9<C>(src, g.plane, fl, rm, r0, rp, xm, (uint32_t)x, xp, d);
        moments9(d, sd, jx, jy);
        rho = rho_off + sd;
        ux = jx / rho;
        uy = jy / rho;
    }
    const size_t o = (size_t)y * g.nx + x;
    if (rho_out) rho_out[o] = rho;
    if (ux_out) ux_out[o] = ux;
    if (uy_out) uy_out[o] = uy;
}

// FP64 reduction of sum u_x, sum rho and the count of bad densities over the
// fluid nodes.  Each block walks a fixed, contiguous range of rows, so the
// partial sums and their final order do not depend on timing.
constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 1024;

__device__ __forceinline__ double block_sum(double v, double *sh) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sh[w];
    return t;
}

template <int S>
__global__ void __launch_bounds__(RED_THREADS) k_reduce(const typename Codec<S>::T *__restrict__ src,
                                                        const uint16_t *__restrict__ flags, Grid g,
                                                        float rho_off, int rows_per_block,
                                                        double *__restrict__ partials) {
    using C = Codec<S>;
    __shared__ double sh[RED_THREADS / 64];
    const uint32_t pitch = (uint32_t)g.pitch;
    double q = 0.0, mass = 0.0, bad = 0.0;
    const int ya = blockIdx.x * rows_per_block, yb = min(ya + rows_per_block, g.ny);
    for (int y = ya; y < yb; ++y) {
        const uint32_t r0 = (uint32_t)y * pitch;
        const uint32_t rm = (uint32_t)(y == 0 ? g.ny - 1 : y - 1) * pitch;
        const uint32_t rp = (uint32_t)(y == g.ny - 1 ? 0 : y + 1) * pitch;
        for (int x = threadIdx.x; x < g.nx; x += blockDim.x) {
            const uint32_t fl = flags[r0 + x];
            if (fl & FL_SOLID) continue;
            const uint32_t xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
            float d[9];
            pull9<C>(src, g.plane, fl, rm, r0, rp, xm, (uint32_t)x, xp, d);
            double rho = (double)rho_off, jx = 0.0;
#pragma unroll
            for (int a = 0; a < 9; ++a) rho += (double)d[a];
            jx = ((double)d[1] - (double)d[3]) + (((double)d[5] - (double)d[7]) + ((double)d[8] - (double)d[6]));
            if (!(rho > 0.0) || !isfinite(rho)) {
                bad += 1.0;
                continue;
            }
            q += jx / rho;
            mass += rho;
        }
    }
    const double tq = block_sum(q, sh);
    const double tm = block_sum(mass, sh);
    const double tb = block_sum(bad, sh);
    if (threadIdx.x == 0) {
        partials[4 * blockIdx.x + 0] = tq;
        partials[4 * blockIdx.x + 1] = tm;
        partials[4 * blockIdx.x + 2] = tb;
        partials[4 * blockIdx.x + 3] = 0.0;
    }
}

// Channel-averaged velocity profile: out[y] = (1/nx) sum over the fluid nodes
// of row y of u_x = j_x / rho (eq. (2)), per node exactly as k_reduce forms it
// (FP64 from the decoded populations); one workgroup per row, fixed tree, so
// the profile sums to the flux of eq. (11) up to the order of the sums.
template <int S>
__global__ void __launch_bounds__(RED_THREADS) k_profile(const typename Codec<S>::T *__restrict__ src,
                                                         const uint16_t *__restrict__ flags, Grid g,
                                                         float rho_off, double inv_nx, double *__restrict__ out) {
    using C = Codec<S>;
    __shared__ double sh[RED_THREADS / 64];
    const uint32_t pitch = (uint32_t)g.pitch;
    const int y = blockIdx.x;
    const uint32_t r0 = (uint32_t)y * pitch;
    const uint32_t rm = (uint32_t)(y == 0 ? g.ny - 1 : y - 1) * pitch;
    const uint32_t rp = (uint32_t)(y == g.ny - 1 ? 0 : y + 1) * pitch;
    double q = 0.0;
    for (int x = threadIdx.x; x < g.nx; x += blockDim.x) {
        const uint32_t fl = flags[r0 + x];
        if (fl & FL_SOLID) continue;
        const uint32_t xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
        float d[9];
        pull9<C>(src, g.plane, fl, rm, r0, rp, xm, (uint32_t)x, xp, d);
        double rho = (double)rho_off;
#pragma unroll
        for (int a = 0; a < 9; ++a) rho += (double)d[a];
        const double jx = ((double)d[1] - (double)d[3]) + (((double)d[5] - (double)d[7]) + ((double)d[8] - (double)d[6]));
        if (rho > 0.0 && isfinite(rho)) q += jx / rho;
    }
    const double t = block_sum(q, sh);
    if (threadIdx.x == 0) out[y] = t * inv_nx;
}

__global__ void __launch_bounds__(64) k_reduce_final(const double *__restrict__ partials, int n,
                                                     double inv_nx, double *__restrict__ out) {
    // lane l sums a contiguous slice in order, lane 0 then sums the 64 slices
    // in order: the same tree for every call
    __shared__ double part[3][64];
    const int l = threadIdx.x;
    const int a = (int)(((int64_t)l * n) / 64), b = (int)(((int64_t)(l + 1) * n) / 64);
    double q = 0.0, mass = 0.0, bad = 0.0;
    for (int k = a; k < b; ++k) {
        q += partials[4 * k + 0];
        mass += partials[4 * k + 1];
        bad += partials[4 * k + 2];
    }
    part[0][l] = q;
    part[1][l] = mass;
    part[2][l] = bad;
    __syncthreads();
    if (l == 0) {
        q = mass = bad = 0.0;
        for (int k = 0; k < 64; ++k) {
            q += part[0][k];
            mass += part[1][k];
            bad += part[2][k];
        }
        out[0] = q * inv_nx;
        out[1] = mass;
        out[2] = bad;
    }
}

// Batched step over many lattices in one persistent launch.  Workgroups pull
// tiles from a queue (one atomic per tile), so uneven channels balance
// dynamically; every channel uses the same tile code as a single lattice.
template <int S, bool TRT, bool SR>
__global__ void __launch_bounds__(512) k_batch_step(const ChannelDesc *__restrict__ descs,
                                                    const uint32_t *__restrict__ tiles,
                                                    uint32_t *__restrict__ counters, int ntiles, int slot,
                                                    int parity, uint32_t *rng) {
    extern __shared__ float ring[];
    __shared__ int next_tile;
    uint32_t mix = 0u;
    if constexpr (SR) mix = sr_step_mix(rng, parity);
    for (;;) {
        if (threadIdx.x == 0) next_tile = (int)atomicAdd(&counters[slot], 1u);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(next_tile);
        __syncthreads();                 // next_tile is rewritten only after all have read it
        if (t >= ntiles) break;
        const uint32_t packed = __builtin_amdgcn_readfirstlane(tiles[t]);
        const ChannelDesc *d = descs + (packed >> 16);
        const Grid g = d->g;
        const Model m = d->m;
        const int chunks = d->chunks;
        const void *src = parity ? d->buf[1] : d->buf[0];
        void *dst = const_cast<void *>(parity ? d->buf[0] : d->buf[1]);
        const int local = (int)(packed & 0xFFFFu);
        const int strip = local / chunks, chunk = local - strip * chunks;
        const int y0 = (int)(((int64_t)chunk * g.ny) / chunks);
        const int y1 = (int)(((int64_t)(chunk + 1) * g.ny) / chunks);
        step_tile<S, TRT, SR>(src, dst, d->flags, d->rowplain, g, m, strip * (int)blockDim.x, y0, y1, (chunk & 1) == 0, ring,
                              mix);
    }
}

// The same batched step with one workgroup per tile (grid = number of tiles,
// tiles mapped to XCDs in contiguous ranges): the hardware dispatcher does the
// balancing and no state is carried between tiles.
template <int S, bool TRT, bool SR>
__global__ void __launch_bounds__(512) k_batch_tiles(const ChannelDesc *__restrict__ descs,
                                                     const uint32_t *__restrict__ tiles, int ntiles,
                                                     int tiles_per_xcd, int parity, uint32_t *rng) {
    extern __shared__ float ring[];
    uint32_t mix = 0u;
    if constexpr (SR) mix = sr_step_mix(rng, parity);
    const int t = (int)(blockIdx.x & 7u) * tiles_per_xcd + (int)(blockIdx.x >> 3);
    if (t >= ntiles) return;
    const uint32_t packed = __builtin_amdgcn_readfirstlane(tiles[t]);
    const ChannelDesc *d = descs + (packed >> 16);
    const Grid g = d->g;
    const Model m = d->m;
    const int chunks = d->chunks;
    const void *src = parity ? d->buf[1] : d->buf[0];
    void *dst = const_cast<void *>(parity ? d->buf[0] : d->buf[1]);
    const int local = (int)(packed & 0xFFFFu);
    const int strip = local / chunks, chunk = local - strip * chunks;
    const int y0 = (int)(((int64_t)chunk * g.ny) / chunks);
    const int y1 = (int)(((int64_t)(chunk + 1) * g.ny) / chunks);
    step_tile<S, TRT, SR>(src, dst, d->flags, d->rowplain, g, m, strip * (int)blockDim.x, y0, y1, (chunk & 1) == 0, ring,
                          mix);
}

// The batched step with K time steps per launch (the multi-step tile of
// k_stepk on every tile of every active channel): one workgroup per tile,
// tiles mapped to XCDs in contiguous ranges, a tile is (channel << 16) |
// (strip * chunks_k + chunk) with strips of BX - 2H output columns.  With
// stochastic rounding the K steps take the step counts count .. count + K - 1
// and the next launch reads count + K, as in k_stepk.
template <int S, bool TRT, bool SR, int BX, int K>
__global__ void __launch_bounds__(BX) k_batch_tilesk(const ChannelDesc *__restrict__ descs,
                                                      const uint32_t *__restrict__ tiles, int ntiles,
                                                      int tiles_per_xcd, int parity, uint32_t *rng) {
    extern __shared__ char ldsk[];
    uint32_t mix[K];
#pragma unroll
    for (int k = 0; k < K; ++k) mix[k] = 0u;
    if constexpr (SR) {
        const uint32_t count = rng[parity];
        if (blockIdx.x == 0 && threadIdx.x == 0) rng[parity ^ 1] = count + (uint32_t)K;
#pragma unroll
        for (int k = 0; k < K; ++k) mix[k] = lowbias32(count + (uint32_t)k + 0x9e3779b9u);
    }
    const int t = (int)(blockIdx.x & 7u) * tiles_per_xcd + (int)(blockIdx.x >> 3);
    if (t >= ntiles) return;        // uniform for the workgroup, before any barrier
    const uint32_t packed = __builtin_amdgcn_readfirstlane(tiles[t]);
    const ChannelDesc *d = descs + (packed >> 16);
    StepArgs a;
    a.src = parity ? d->buf[1] : d->buf[0];
    a.dst = const_cast<void *>(parity ? d->buf[0] : d->buf[1]);
    a.flags = d->flags;
    a.g = d->g;
    a.m = d->m;
    const int chunks = d->chunks_k;
    const int local = (int)(packed & 0xFFFFu);
    const int strip = local / chunks, chunk = local - strip * chunks;
    const int y0 = (int)(((int64_t)chunk * a.g.ny) / chunks);
    const int y1 = (int)(((int64_t)(chunk + 1) * a.g.ny) / chunks);
    stepk_tile<S, TRT, SR, BX, K>(a, strip * (BX - 2 * Multi<K>::H), y0, y1, (chunk & 1) == 0, ldsk, mix);
}

// Per-channel FP64 flux/mass reduction: one workgroup per channel, rows in
// order, fixed reduction tree (bitwise reproducible).
template <int S>
__global__ void __launch_bounds__(256) k_batch_reduce(const ChannelDesc *__restrict__ descs,
                                                      const int32_t *__restrict__ ids,
                                                      const int32_t *__restrict__ cur,
                                                      double *__restrict__ out) {
    using C = Codec<S>;
    __shared__ double sh[4];
    const int id = ids[blockIdx.x];
    const ChannelDesc d = descs[id];
    const Grid g = d.g;
    const typename C::T *src = static_cast<const typename C::T *>(d.buf[cur[id]]);
    const uint32_t pitch = (uint32_t)g.pitch;
    double q = 0.0, mass = 0.0, bad = 0.0;
    for (int y = 0; y < g.ny; ++y) {
        const uint32_t r0 = (uint32_t)y * pitch;
        const uint32_t rm = (uint32_t)(y == 0 ? g.ny - 1 : y - 1) * pitch;
        const uint32_t rp = (uint32_t)(y == g.ny - 1 ? 0 : y + 1) * pitch;
        for (int x = threadIdx.x; x < g.nx; x += blockDim.x) {
            const uint32_t fl = d.flags[r0 + x];
            if (fl & FL_SOLID) continue;
            const uint32_t xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
            float v[9];
            pull9<C>(src, g.plane, fl, rm, r0, rp, xm, (uint32_t)x, xp, v);
            double rho = (double)d.m.rho_off;
#pragma unroll
            for (int k = 0; k < 9; ++k) rho += (double)v[k];
            const double jx = ((double)v[1] - (double)v[3]) +
                              (((double)v[5] - (double)v[7]) + ((double)v[8] - (double)v[6]));
            if (!(rho > 0.0) || !isfinite(rho)) {
                bad += 1.0;
                continue;
            }
            q += jx / rho;
            mass += rho;
        }
    }
    const double tq = block_sum(q, sh);
    const double tm = block_sum(mass, sh);
    const double tb = block_sum(bad, sh);
    if (threadIdx.x == 0) {
        out[4 * blockIdx.x + 0] = tq / (double)g.nx;
        out[4 * blockIdx.x + 1] = tm;
        out[4 * blockIdx.x + 2] = tb;
        out[4 * blockIdx.x + 3] = 0.0;
    }
}

}  // namespace

// The fused step kernel for (storage, collision, rounding); null for
// stochastic rounding of FP32 data (not instantiated).
using StepKernel = void (*)(const StepArgs);
template <bool EIGHT, int S, bool TRT, bool SR>
StepKernel step_k() {
    if constexpr (EIGHT) return k_step8<S, TRT, SR>;
    else return k_step<S, TRT, SR>;
}
template <bool EIGHT, int S>
StepKernel step_k16(bool trt, bool sr) {
    return trt ? (sr ? step_k<EIGHT, S, true, true>() : step_k<EIGHT, S, true, false>())
               : (sr ? step_k<EIGHT, S, false, true>() : step_k<EIGHT, S, false, false>());
}
template <bool EIGHT>
StepKernel step_kernel(int storage, bool trt, bool sr) {
    switch (storage) {
    case ST_F32:
        if (sr) return nullptr;
        return trt ? step_k<EIGHT, ST_F32, true, false>() : step_k<EIGHT, ST_F32, false, false>();
    case ST_F16: return step_k16<EIGHT, ST_F16>(trt, sr);
    case ST_BF16: return step_k16<EIGHT, ST_BF16>(trt, sr);
    default: return nullptr;
    }
}

template <bool EIGHT>
hipError_t launch_step_k(int storage, const StepArgs &a, int block_x, hipStream_t s) {
    StepKernel k = step_kernel<EIGHT>(storage, a.m.trt != 0, a.m.sround != 0);
    if (a.acc) {            // fused kernel, paper operator, nearest rounding only (checked by the host)
        if (EIGHT || a.m.trt || a.m.sround) return hipErrorInvalidValue;
        k = storage == ST_F32 ? k_step_acc<ST_F32> : storage == ST_F16 ? k_step_acc<ST_F16>
                                                                       : k_step_acc<ST_BF16>;
    }
    if (!k) return hipErrorInvalidValue;
    const unsigned blocks = 8u * (unsigned)a.tiles_per_xcd;
    const size_t lds = (size_t)RING * (block_x + 2) * sizeof(float);
    k<<<blocks, block_x, lds, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_step(int storage, const StepArgs &a, int block_x, hipStream_t s) {
    return launch_step_k<false>(storage, a, block_x, s);
}

// The multi-step kernels are compiled for K = 2, 3 steps per launch and
// block_x 256 and 512 (ring strides are compile-time constants).
template <int S, int BX, int K>
StepKernel stepk_k16(bool trt, bool sr) {
    return trt ? (sr ? k_stepk<S, true, true, BX, K> : k_stepk<S, true, false, BX, K>)
               : (sr ? k_stepk<S, false, true, BX, K> : k_stepk<S, false, false, BX, K>);
}
template <int BX, int K>
StepKernel stepk_kernel_bx(int storage, bool trt, bool sr) {
    switch (storage) {
    case ST_F32:
        if (sr) return nullptr;
        return trt ? k_stepk<ST_F32, true, false, BX, K> : k_stepk<ST_F32, false, false, BX, K>;
    case ST_F16: return stepk_k16<ST_F16, BX, K>(trt, sr);
    case ST_BF16: return stepk_k16<ST_BF16, BX, K>(trt, sr);
    default: return nullptr;
    }
}
template <int K>
StepKernel stepk_kernel_k(int storage, int block_x, bool trt, bool sr) {
    switch (block_x) {
    case 256: return stepk_kernel_bx<256, K>(storage, trt, sr);
    case 512: return stepk_kernel_bx<512, K>(storage, trt, sr);
    default: return nullptr;
    }
}
StepKernel stepk_kernel(int storage, int block_x, int k, bool trt, bool sr) {
    switch (k) {
    case 2: return stepk_kernel_k<2>(storage, block_x, trt, sr);
    case 3: return stepk_kernel_k<3>(storage, block_x, trt, sr);
    default: return nullptr;
    }
}
size_t stepk_lds_bytes(int storage, int block_x, int k) {
    if (k == 3) return storage == ST_F32 ? multi_lds_bytes<ST_F32, 3>(block_x) : multi_lds_bytes<ST_F16, 3>(block_x);
    return storage == ST_F32 ? multi_lds_bytes<ST_F32, 2>(block_x) : multi_lds_bytes<ST_F16, 2>(block_x);
}

hipError_t launch_stepk(int storage, const StepArgs &a, int block_x, int k, hipStream_t s) {
    StepKernel kern = stepk_kernel(storage, block_x, k, a.m.trt != 0, a.m.sround != 0);
    if (!kern || a.acc) return hipErrorInvalidValue;
    const unsigned blocks = 8u * (unsigned)a.tiles_per_xcd;
    kern<<<blocks, block_x, stepk_lds_bytes(storage, block_x, k), s>>>(a);
    return hipGetLastError();
}

int stepk_blocks_per_cu(int storage, int block_x, int k, bool trt, bool sr) {
    StepKernel kern = stepk_kernel(storage, block_x, k, trt, sr);
    if (!kern) return 1;
    int n = 0;
    const hipError_t e =
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, block_x, stepk_lds_bytes(storage, block_x, k));
    return e == hipSuccess && n > 0 ? n : 1;
}

hipError_t launch_step8(int storage, const StepArgs &a, int block_x, hipStream_t s) {
    return launch_step_k<true>(storage, a, block_x, s);
}

template <int V>
hipError_t launch_wide_v(int storage, const StepArgs &a, int block_x, hipStream_t s) {
    const unsigned blocks = 8u * (unsigned)a.tiles_per_xcd;
    const size_t lds = (size_t)RING * (block_x * V + 2) * sizeof(float);
    switch (storage) {
    case ST_F32: k_step_wide<ST_F32, V><<<blocks, block_x, lds, s>>>(a); break;
    case ST_F16: k_step_wide<ST_F16, V><<<blocks, block_x, lds, s>>>(a); break;
    case ST_BF16: k_step_wide<ST_BF16, V><<<blocks, block_x, lds, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step_wide(int storage, const StepArgs &a, int block_x, int v, hipStream_t s) {
    switch (v) {
    case 2: return launch_wide_v<2>(storage, a, block_x, s);
    case 4: return launch_wide_v<4>(storage, a, block_x, s);
    default: return hipErrorInvalidValue;
    }
}

template <int V>
int wide_blocks_v(int storage, int block_x) {
    const size_t lds = (size_t)RING * (block_x * V + 2) * sizeof(float);
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (storage) {
    case ST_F32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_wide<ST_F32, V>, block_x, lds); break;
    case ST_F16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_wide<ST_F16, V>, block_x, lds); break;
    case ST_BF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_wide<ST_BF16, V>, block_x, lds); break;
    default: break;
    }
    return e == hipSuccess && n > 0 ? n : 1;
}

int wide_blocks_per_cu(int storage, int block_x, int v) {
    return v == 4 ? wide_blocks_v<4>(storage, block_x) : wide_blocks_v<2>(storage, block_x);
}

template <int BX>
hipError_t launch_split_bx(int storage, const StepArgs &a, hipStream_t s) {
    const unsigned blocks = 8u * (unsigned)a.tiles_per_xcd;
    switch (storage) {
    case ST_F32: k_step_split<ST_F32, BX><<<blocks, BX + 64, 0, s>>>(a); break;
    case ST_F16: k_step_split<ST_F16, BX><<<blocks, BX + 64, 0, s>>>(a); break;
    case ST_BF16: k_step_split<ST_BF16, BX><<<blocks, BX + 64, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step_split(int storage, const StepArgs &a, int block_x, hipStream_t s) {
    switch (block_x) {
    case 128: return launch_split_bx<128>(storage, a, s);
    case 256: return launch_split_bx<256>(storage, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int BX>
int split_blocks_bx(int storage) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (storage) {
    case ST_F32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_split<ST_F32, BX>, BX + 64, 0); break;
    case ST_F16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_split<ST_F16, BX>, BX + 64, 0); break;
    case ST_BF16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_step_split<ST_BF16, BX>, BX + 64, 0); break;
    default: break;
    }
    return e == hipSuccess && n > 0 ? n : 1;
}

int split_blocks_per_cu(int storage, int block_x) {
    return block_x == 128 ? split_blocks_bx<128>(storage) : split_blocks_bx<256>(storage);
}

template <bool EIGHT>
int step_k_blocks_per_cu(int storage, int block_x, bool trt, bool sr) {
    const StepKernel k = step_kernel<EIGHT>(storage, trt, sr);
    if (!k) return 1;
    const size_t lds = (size_t)RING * (block_x + 2) * sizeof(float);
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block_x, lds);
    return e == hipSuccess && n > 0 ? n : 1;
}

int step_blocks_per_cu(int storage, int block_x, bool trt, bool sr) {
    return step_k_blocks_per_cu<false>(storage, block_x, trt, sr);
}

int step8_blocks_per_cu(int storage, int block_x, bool trt, bool sr) {
    return step_k_blocks_per_cu<true>(storage, block_x, trt, sr);
}

hipError_t launch_init(int storage, void *dst, const uint16_t *flags, const Grid &g, float off,
                       const float *rho, const float *ux, const float *uy, int dense_pitch,
                       hipStream_t s) {
    const dim3 grid((g.nx + 255) / 256, g.ny);
    switch (storage) {
    case ST_F32:
        k_init<ST_F32><<<grid, 256, 0, s>>>((float *)dst, flags, g, rho, ux, uy, dense_pitch, off);
        break;
    case ST_F16:
        k_init<ST_F16><<<grid, 256, 0, s>>>((_Float16 *)dst, flags, g, rho, ux, uy, dense_pitch, off);
        break;
    case ST_BF16:
        k_init<ST_BF16><<<grid, 256, 0, s>>>((__bf16 *)dst, flags, g, rho, ux, uy, dense_pitch, off);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_fill(void *dst, size_t bytes, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t blocks = (n16 + 255) / 256;
    k_fill<<<(unsigned)(blocks < 8192 ? blocks : 8192), 256, 0, s>>>((uint4 *)dst, n16);
    return hipGetLastError();
}

// The 16-bit stochastic rounding of the step kernels' stores, value by value
// (Codec<S>::enc_sr), for tests of the encoder itself.
template <int S>
__global__ void __launch_bounds__(256) k_round_sr(const float *__restrict__ in, const uint32_t *__restrict__ r,
                                                  uint16_t *__restrict__ out, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = __builtin_bit_cast(uint16_t, Codec<S>::enc_sr(in[i], r[i]));
}

hipError_t launch_round_sr(const float *in, const uint32_t *r, uint16_t *out, uint32_t n, int storage,
                           hipStream_t s) {
    if (n == 0) return hipSuccess;
    const unsigned blocks = (n + 255u) / 256u;
    if (storage == ST_F16) k_round_sr<ST_F16><<<blocks, 256, 0, s>>>(in, r, out, n);
    else if (storage == ST_BF16) k_round_sr<ST_BF16><<<blocks, 256, 0, s>>>(in, r, out, n);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, int per_lane, hipStream_t s) {
    const size_t n16 = bytes / 16;
    if (n16 == 0) return hipSuccess;
    const size_t per_block = (size_t)256 * per_lane;
    const size_t blocks = (n16 + per_block - 1) / per_block;
    if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
    switch (per_lane) {
    case 1: k_stream_copy<1><<<(unsigned)blocks, 256, 0, s>>>((v4u *)dst, (const v4u *)src, n16); break;
    case 2: k_stream_copy<2><<<(unsigned)blocks, 256, 0, s>>>((v4u *)dst, (const v4u *)src, n16); break;
    case 4: k_stream_copy<4><<<(unsigned)blocks, 256, 0, s>>>((v4u *)dst, (const v4u *)src, n16); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_moments(int storage, const void *src, const uint16_t *flags, const Grid &g,
                          float rho_off, float *rho, float *ux, float *uy, hipStream_t s) {
    const dim3 grid((g.nx + 255) / 256, g.ny);
    switch (storage) {
    case ST_F32: k_moments<ST_F32><<<grid, 256, 0, s>>>((const float *)src, flags, g, rho_off, rho, ux, uy); break;
    case ST_F16: k_moments<ST_F16><<<grid, 256, 0, s>>>((const _Float16 *)src, flags, g, rho_off, rho, ux, uy); break;
    case ST_BF16: k_moments<ST_BF16><<<grid, 256, 0, s>>>((const __bf16 *)src, flags, g, rho_off, rho, ux, uy); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int max_reduce_blocks() { return RED_MAX_BLOCKS; }

hipError_t launch_profile(int storage, const void *src, const uint16_t *flags, const Grid &g, float rho_off,
                          double *out, hipStream_t s) {
    const double inv_nx = 1.0 / (double)g.nx;
    switch (storage) {
    case ST_F32: k_profile<ST_F32><<<g.ny, RED_THREADS, 0, s>>>((const float *)src, flags, g, rho_off, inv_nx, out); break;
    case ST_F16: k_profile<ST_F16><<<g.ny, RED_THREADS, 0, s>>>((const _Float16 *)src, flags, g, rho_off, inv_nx, out); break;
    case ST_BF16: k_profile<ST_BF16><<<g.ny, RED_THREADS, 0, s>>>((const __bf16 *)src, flags, g, rho_off, inv_nx, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Rows per workgroup of the FP64 reduction (at most RED_MAX_BLOCKS workgroups).
int reduce_rows(const Grid &g) { return std::max(1, (g.ny + RED_MAX_BLOCKS - 1) / RED_MAX_BLOCKS); }

int reduce_blocks(const Grid &g) {
    const int rows = reduce_rows(g);
    return (g.ny + rows - 1) / rows;
}

hipError_t launch_reduce(int storage, const void *src, const uint16_t *flags, const Grid &g,
                         float rho_off, double *partials, double *out, hipStream_t s) {
    const int rows = reduce_rows(g);
    const int blocks = (g.ny + rows - 1) / rows;
    switch (storage) {
    case ST_F32: k_reduce<ST_F32><<<blocks, RED_THREADS, 0, s>>>((const float *)src, flags, g, rho_off, rows, partials); break;
    case ST_F16: k_reduce<ST_F16><<<blocks, RED_THREADS, 0, s>>>((const _Float16 *)src, flags, g, rho_off, rows, partials); break;
    case ST_BF16: k_reduce<ST_BF16><<<blocks, RED_THREADS, 0, s>>>((const __bf16 *)src, flags, g, rho_off, rows, partials); break;
    default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reduce_final<<<1, 64, 0, s>>>(partials, blocks, 1.0 / (double)g.nx, out);
    return hipGetLastError();
}


// Batch kernels for (storage, collision, rounding), as for the single lattice.
using BatchTilesKernel = void (*)(const ChannelDesc *, const uint32_t *, int, int, int, uint32_t *);
using BatchQueueKernel = void (*)(const ChannelDesc *, const uint32_t *, uint32_t *, int, int, int, uint32_t *);
template <bool QUEUE, int S, bool TRT, bool SR>
auto batch_k() {
    if constexpr (QUEUE) return k_batch_step<S, TRT, SR>;
    else return k_batch_tiles<S, TRT, SR>;
}
template <bool QUEUE, int S>
auto batch_k16(bool trt, bool sr) {
    return trt ? (sr ? batch_k<QUEUE, S, true, true>() : batch_k<QUEUE, S, true, false>())
               : (sr ? batch_k<QUEUE, S, false, true>() : batch_k<QUEUE, S, false, false>());
}
template <bool QUEUE>
auto batch_kernel(int storage, bool trt, bool sr) -> decltype(batch_k<QUEUE, ST_F32, false, false>()) {
    switch (storage) {
    case ST_F32:
        if (sr) return nullptr;
        return trt ? batch_k<QUEUE, ST_F32, true, false>() : batch_k<QUEUE, ST_F32, false, false>();
    case ST_F16: return batch_k16<QUEUE, ST_F16>(trt, sr);
    case ST_BF16: return batch_k16<QUEUE, ST_BF16>(trt, sr);
    default: return nullptr;
    }
}

hipError_t launch_batch_step(int storage, const BatchStepArgs &a, int block_x, int grid, hipStream_t s) {
    const size_t lds = (size_t)RING * (block_x + 2) * sizeof(float);
    const bool trt = a.trt != 0, sr = a.sround != 0;
    if (grid <= 0) {   // one workgroup per tile
        const BatchTilesKernel k = batch_kernel<false>(storage, trt, sr);
        if (!k) return hipErrorInvalidValue;
        const int per = (a.ntiles + 7) / 8;
        k<<<8 * per, block_x, lds, s>>>(a.descs, a.tiles, a.ntiles, per, a.parity, a.rng);
        return hipGetLastError();
    }
    const BatchQueueKernel k = batch_kernel<true>(storage, trt, sr);
    if (!k) return hipErrorInvalidValue;
    k<<<grid, block_x, lds, s>>>(a.descs, a.tiles, a.counters, a.ntiles, a.slot, a.parity, a.rng);
    return hipGetLastError();
}

int batch_blocks_per_cu(int storage, int block_x, bool trt, bool sr) {
    const BatchQueueKernel k = batch_kernel<true>(storage, trt, sr);
    if (!k) return 1;
    const size_t lds = (size_t)RING * (block_x + 2) * sizeof(float);
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, block_x, lds);
    return e == hipSuccess && n > 0 ? n : 1;
}

using BatchTilesKKernel = void (*)(const ChannelDesc *, const uint32_t *, int, int, int, uint32_t *);
template <int S, int BX, int K>
BatchTilesKKernel batchk_k16(bool trt, bool sr) {
    return trt ? (sr ? k_batch_tilesk<S, true, true, BX, K> : k_batch_tilesk<S, true, false, BX, K>)
               : (sr ? k_batch_tilesk<S, false, true, BX, K> : k_batch_tilesk<S, false, false, BX, K>);
}
template <int BX, int K>
BatchTilesKKernel batchk_kernel_bx(int storage, bool trt, bool sr) {
    switch (storage) {
    case ST_F32:
        if (sr) return nullptr;
        return trt ? k_batch_tilesk<ST_F32, true, false, BX, K> : k_batch_tilesk<ST_F32, false, false, BX, K>;
    case ST_F16: return batchk_k16<ST_F16, BX, K>(trt, sr);
    case ST_BF16: return batchk_k16<ST_BF16, BX, K>(trt, sr);
    default: return nullptr;
    }
}
template <int K>
BatchTilesKKernel batchk_kernel_k(int storage, int block_x, bool trt, bool sr) {
    switch (block_x) {
    case 256: return batchk_kernel_bx<256, K>(storage, trt, sr);
    case 512: return batchk_kernel_bx<512, K>(storage, trt, sr);
    default: return nullptr;
    }
}

hipError_t launch_batch_stepk(int storage, const BatchStepArgs &a, int block_x, int k, hipStream_t s) {
    BatchTilesKKernel kern = k == 2 ? batchk_kernel_k<2>(storage, block_x, a.trt != 0, a.sround != 0)
                           : k == 3 ? batchk_kernel_k<3>(storage, block_x, a.trt != 0, a.sround != 0)
                                    : nullptr;
    if (!kern) return hipErrorInvalidValue;
    const int per = (a.ntiles + 7) / 8;
    kern<<<8 * per, block_x, stepk_lds_bytes(storage, block_x, k), s>>>(a.descs, a.tiles, a.ntiles, per, a.parity,
                                                                       a.rng);
    return hipGetLastError();
}

hipError_t launch_batch_reduce(int storage, const ChannelDesc *descs, const int32_t *ids,
                               const int32_t *cur, int n, double *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (storage) {
    case ST_F32: k_batch_reduce<ST_F32><<<n, 256, 0, s>>>(descs, ids, cur, out); break;
    case ST_F16: k_batch_reduce<ST_F16><<<n, 256, 0, s>>>(descs, ids, cur, out); break;
    case ST_BF16: k_batch_reduce<ST_BF16><<<n, 256, 0, s>>>(descs, ids, cur, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lbm
