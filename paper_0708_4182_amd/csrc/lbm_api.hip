// Host side of liblbm: the C ABI declared in include/lbm.h.
//
// Validates parameters, derives the per-node flag words from the solid mask
// (integer arithmetic on the host), carves the caller's device workspace into
// two population buffers, the flags and reduction scratch, and issues the
// kernels of lbm_kernels.hip on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using lbm::Grid;
using lbm::Model;

struct lbm_sim {
    lbm_params p{};
    Grid g{};
    Model m{};
    hipStream_t stream = nullptr;
    int device = 0;
    char *buf[2] = {nullptr, nullptr};
    size_t buf_bytes = 0;
    uint16_t *flags = nullptr;
    double *partials = nullptr;
    double *result = nullptr;
    uint32_t *rowplain = nullptr;   // rows whose flag words are all plain (one bit per row)
    uint32_t *rng = nullptr;   // two-slot step counter of stochastic rounding
    uint32_t rng_host[2] = {0u, 0u};
    const float *acc = nullptr;         // per-node acceleration field [2][ny][nx] (caller's device memory)
    double *static_scratch = nullptr;   // this device's copy of the library's static scratch (lbm_flux_static)
    std::string static_err;             // why static_scratch is NULL, if it is
    int cur = 0;
    int64_t steps = 0;
    int block_x = 256;
    int rows = 0;          // rows per chunk; 0 = one wave of resident workgroups
    int kernel = LBM_KERNEL_FUSED;
    int cus = 0;           // compute units of the device
    int max_lds = 0;       // LDS bytes one workgroup may use on the device
    int chunks = 0;        // cached tiling (0 = recompute)
    int chunks1 = 0;       // cached tiling of the fused kernel, which runs the remainder steps of a multi-step kernel
    int graph_steps = 0;   // steps per hipGraph replay (0: eager launches only)
    hipStream_t cap = nullptr;                  // private stream used only for graph capture
    hipGraph_t graph[2] = {nullptr, nullptr};   // per source-buffer parity
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    lbm_status sticky = LBM_OK;
    std::string err;
};

// Device scratch of lbm_flux_static: the FP64 partial sums of the reduction
// (4 doubles per workgroup, at most lbm::max_reduce_blocks() workgroups) and
// the 3-double result, in a file-scope device array instead of the caller's
// workspace.  Each device holds its own copy until the process ends; host code
// uses only the address hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticPartials = 4 * 1024;
constexpr size_t kStaticDoubles = kStaticPartials + 32;   // partials, then the result (256-byte aligned)
static __device__ __align__(256) double scratch[kStaticDoubles];

namespace {

thread_local std::string g_init_error;

// Address of `scratch` on the current device, looked up once per device (the
// first lbm_init on it) and kept; NULL with a message if the lookup failed.
std::mutex g_scratch_mu;
std::map<int, double *> g_scratch_ptr;

double *static_scratch_on(int device, std::string &why) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        why = std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e);
        return nullptr;                 // not cached: a later lbm_init on this device tries again
    }
    g_scratch_ptr[device] = (double *)ptr;
    return (double *)ptr;
}

constexpr size_t kAlign = 256;
constexpr uint64_t kStateMagic = 0x314d54534d424c00ull;  // "\0LBMSTM1"

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int storage) { return storage == LBM_F32 ? 4 : 2; }

struct Layout {
    Grid g;
    size_t buf_bytes, flags_off, flags_bytes, rowplain_off, part_off, res_off, rng_off, total;
    size_t buf_off[2];
};

bool finite_all(const lbm_params *p) {
    const double v[] = {p->tau, p->rho0, p->g_axis, p->g_diag, p->w_axis, p->w_diag,
                        p->rho_c, p->f_elec, p->accel_x, p->accel_y, p->rho_ref, p->trt_magic};
    for (double d : v)
        if (!std::isfinite(d)) return false;
    return true;
}

// Returns an empty string if the parameters are valid, else the reason.
std::string check_params(const lbm_params *p) {
    if (!p) return "params is NULL";
    if (p->nx < 3 || p->ny < 3) return "nx and ny must be >= 3";
    if (!finite_all(p)) return "parameters must be finite";
    if (!(p->tau > 0.5)) return "tau must be > 0.5";
    if (!(p->rho0 > 0.0)) return "rho0 must be > 0";
    if (!(p->rho_ref >= 0.0)) return "rho_ref must be >= 0";
    if (p->storage < LBM_F32 || p->storage > LBM_BF16) return "storage must be LBM_F32, LBM_F16 or LBM_BF16";
    if (p->elec_layers < 0 || p->elec_layers > 1024) return "elec_layers must be in [0, 1024]";
    if (p->elec_walls > 3u) return "elec_walls must be a combination of LBM_ELEC_BOTTOM and LBM_ELEC_TOP";
    if (p->collision != LBM_COLLIDE_BGK && p->collision != LBM_COLLIDE_TRT_GUO &&
        p->collision != LBM_COLLIDE_MRT_GUO)
        return "collision must be LBM_COLLIDE_BGK, LBM_COLLIDE_TRT_GUO or LBM_COLLIDE_MRT_GUO";
    if (p->collision != LBM_COLLIDE_BGK && !(p->trt_magic > 0.0)) return "trt_magic must be > 0";
    if (p->collision == LBM_COLLIDE_MRT_GUO &&
        !(p->mrt_s_e > 0.0 && p->mrt_s_e < 2.0 && p->mrt_s_eps > 0.0 && p->mrt_s_eps < 2.0))
        return "mrt_s_e and mrt_s_eps must be in (0, 2)";
    if (p->elec_normal != 0 && p->elec_normal != 1) return "elec_normal must be 0 or 1";
    if (p->rounding != LBM_ROUND_NEAREST && p->rounding != LBM_ROUND_STOCHASTIC)
        return "rounding must be LBM_ROUND_NEAREST or LBM_ROUND_STOCHASTIC";
    if (p->rounding == LBM_ROUND_STOCHASTIC && p->storage == LBM_F32)
        return "LBM_ROUND_STOCHASTIC needs LBM_F16 or LBM_BF16 storage";
    return "";
}

bool make_layout(const lbm_params *p, Layout &L) {
    if (!check_params(p).empty()) return false;
    L.g.nx = p->nx;
    L.g.ny = p->ny;
    L.g.pitch = (int32_t)align_up((size_t)p->nx, 64);
    const size_t plane = (size_t)L.g.pitch * (size_t)p->ny;
    L.buf_bytes = align_up(9 * plane * elem_size(p->storage), kAlign);
    // 32-bit byte offsets inside one population buffer
    if (9 * plane * elem_size(p->storage) >= (size_t(1) << 32)) return false;
    // the init staging (3 float32 planes) lives in the spare population buffer
    if (3 * (size_t)p->nx * p->ny * sizeof(float) > L.buf_bytes) return false;
    L.g.plane = (uint32_t)plane;
    L.buf_off[0] = 0;
    L.buf_off[1] = L.buf_bytes;
    L.flags_off = 2 * L.buf_bytes;
    L.flags_bytes = align_up(plane * sizeof(uint16_t), kAlign);
    L.rowplain_off = L.flags_off + L.flags_bytes;
    L.part_off = L.rowplain_off + align_up(sizeof(uint32_t) * (size_t)((p->ny + 31) / 32), kAlign);
    L.res_off = L.part_off + align_up(4 * sizeof(double) * (size_t)lbm::max_reduce_blocks(), kAlign);
    L.rng_off = L.res_off + kAlign;
    L.total = L.rng_off + kAlign;
    return true;
}

// Reference density of the stored deviations (lbm_params.rho_ref, else the
// format's default).
float storage_offset(const lbm_params *p) {
    if (p->rho_ref > 0.0) return (float)p->rho_ref;
    return p->storage == LBM_F32 ? 0.f : (float)p->rho0;
}

Model make_model(const lbm_params *p) {
    Model m;
    m.tau = (float)p->tau;
    m.omega = (float)(1.0 / p->tau);
    m.rho0 = (float)p->rho0;
    m.log2e_inv_rho0 = (float)(1.0 / (p->rho0 * std::log(2.0)));
    m.rho_off = storage_offset(p);
    m.ga = (float)p->g_axis;
    m.gd = (float)p->g_diag;
    m.wa = (float)p->w_axis;
    m.wd = (float)p->w_diag;
    m.rho_c = (float)p->rho_c;
    m.f_elec = (float)p->f_elec;
    m.f_elec_diag = (float)(p->f_elec / std::sqrt(2.0));
    m.gx = (float)p->accel_x;
    m.gy = (float)p->accel_y;
    m.trt = p->collision == LBM_COLLIDE_TRT_GUO ? 1 : p->collision == LBM_COLLIDE_MRT_GUO ? 2 : 0;
    m.mrt_se = (float)(p->collision == LBM_COLLIDE_MRT_GUO ? p->mrt_s_e : 0.0);
    m.mrt_seps = (float)(p->collision == LBM_COLLIDE_MRT_GUO ? p->mrt_s_eps : 0.0);
    const double om_m = m.trt ? 1.0 / (p->trt_magic / (p->tau - 0.5) + 0.5) : 1.0 / p->tau;
    m.omega_m = (float)om_m;
    m.src_p = (float)(1.0 - 0.5 / p->tau);
    m.src_m = (float)(1.0 - 0.5 * om_m);
    m.sround = p->rounding == LBM_ROUND_STOCHASTIC ? 1 : 0;
    return m;
}

// Flag words (see lbm_geometry in lbm.h).  The electric layer is the set of
// fluid nodes whose Chebyshev distance to a solid node is <= elec_layers, on
// the half of the domain next to an electrode wall; the Chebyshev ball is a
// square, so the test is a separable max-filter along x then along y.
void derive_flags(const lbm_params *p, const uint8_t *solid, std::vector<uint16_t> &out) {
    const int nx = p->nx, ny = p->ny;
    const int k = p->elec_layers;
    auto S = [&](int x, int y) -> int {
        x %= nx; if (x < 0) x += nx;
        y %= ny; if (y < 0) y += ny;
        return solid[(size_t)y * nx + x] ? 1 : 0;
    };
    std::vector<uint8_t> near((size_t)nx * ny, 0);
    if (k > 0) {
        std::vector<uint8_t> rowmax((size_t)nx * ny, 0);
        const int kx = std::min(k, nx), ky = std::min(k, ny);
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                uint8_t v = 0;
                for (int d = -kx; d <= kx && !v; ++d) v = (uint8_t)S(x + d, y);
                rowmax[(size_t)y * nx + x] = v;
            }
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                uint8_t v = 0;
                for (int d = -ky; d <= ky && !v; ++d) {
                    int yy = (y + d) % ny; if (yy < 0) yy += ny;
                    v = rowmax[(size_t)yy * nx + x];
                }
                near[(size_t)y * nx + x] = v;
            }
    }
    // e_1..e_8
    static const int ex[8] = {1, 0, -1, 0, 1, -1, -1, 1};
    static const int ey[8] = {0, 1, 0, -1, 1, 1, -1, -1};
    // direction a (1..8) of the electric force along the local face normal:
    // sign of the summed displacements to the nearest solid nodes (Chebyshev
    // distance), 0 where they cancel
    auto normal_code = [&](int x, int y) -> uint32_t {
        int dmin = k + 1;
        for (int dy = -k; dy <= k; ++dy)
            for (int dx = -k; dx <= k; ++dx)
                if (S(x + dx, y + dy)) dmin = std::min(dmin, std::max(std::abs(dx), std::abs(dy)));
        long vx = 0, vy = 0;
        for (int dy = -dmin; dy <= dmin; ++dy)
            for (int dx = -dmin; dx <= dmin; ++dx)
                if (std::max(std::abs(dx), std::abs(dy)) == dmin && S(x + dx, y + dy)) { vx += dx; vy += dy; }
        const int sx = (vx > 0) - (vx < 0), sy = (vy > 0) - (vy < 0);
        for (int b = 0; b < 8; ++b)
            if (ex[b] == sx && ey[b] == sy) return (uint32_t)(b + 1);
        return 0u;
    };
    out.assign((size_t)nx * ny, 0);
    for (int y = 0; y < ny; ++y) {
        const bool top = y >= ny / 2;
        const bool electrode = (p->elec_walls & (top ? LBM_ELEC_TOP : LBM_ELEC_BOTTOM)) != 0;
        for (int x = 0; x < nx; ++x) {
            const size_t i = (size_t)y * nx + x;
            if (solid[i]) { out[i] = (uint16_t)lbm::FL_SOLID; continue; }
            uint32_t v = 0;
            for (int b = 0; b < 8; ++b)
                if (S(x + ex[b], y + ey[b])) v |= 1u << b;
            if (electrode && near[i]) {
                v |= lbm::FL_LAYER;
                if (p->elec_normal) v |= normal_code(x, y) << lbm::FL_NSHIFT;
            }
            if (top) v |= lbm::FL_TOP;
            out[i] = (uint16_t)v;
        }
    }
}

lbm_status fail(lbm_sim *s, lbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (s) {
        s->err = buf;
        if (st != LBM_EINVAL) s->sticky = st;
    } else {
        g_init_error = buf;
    }
    return st;
}

#define HIP_TRY(sim, expr)                                                                      \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail((sim), LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess || prev == dev || hipSetDevice(dev) != hipSuccess) prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

lbm_status usable(lbm_sim *s) {
    if (!s) return LBM_EINVAL;
    if (s->sticky != LBM_OK) return LBM_ESTATE;
    return LBM_OK;
}

lbm_status do_flux(lbm_sim *s, double *Q, double *M, double *partials, double *result) {
    HIP_TRY(s, lbm::launch_reduce(s->p.storage, s->buf[s->cur], s->flags, s->g, s->m.rho_off,
                                  partials, result, s->stream));
    double host[3];
    HIP_TRY(s, hipMemcpyAsync(host, result, sizeof host, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    if (Q) *Q = host[0];
    if (M) *M = host[1];
    if (host[2] != 0.0)
        return fail(s, LBM_EDIVERGED, "%.0f fluid nodes have a density <= 0 or not finite after %lld steps",
                    host[2], (long long)s->steps);
    return LBM_OK;
}

}  // namespace

namespace lbm {
std::string check_params_str(const lbm_params *p) { return check_params(p); }
Model make_model_of(const lbm_params *p) { return make_model(p); }
float storage_offset_of(const lbm_params *p) { return storage_offset(p); }
void derive_flags_of(const lbm_params *p, const uint8_t *solid, std::vector<uint16_t> &out) {
    derive_flags(p, solid, out);
}
// Bit y (word y / 32) set when every node of row y has the plain flag word:
// 0 below ny / 2, FL_TOP from there (a fluid node with no solid neighbour
// outside the electric layer).  The step kernel then skips that row's flags.
void row_plain_mask(int nx, int ny, const std::vector<uint16_t> &fl, std::vector<uint32_t> &mask) {
    mask.assign((size_t)(ny + 31) / 32, 0u);
    for (int y = 0; y < ny; ++y) {
        const uint16_t plain = (uint16_t)(y >= ny / 2 ? lbm::FL_TOP : 0u);
        bool all = true;
        for (int x = 0; x < nx && all; ++x) all = fl[(size_t)y * nx + x] == plain;
        if (all) mask[(size_t)y / 32] |= 1u << (y % 32);
    }
}
}  // namespace lbm

extern "C" {

size_t lbm_workspace_bytes(const lbm_params *p) {
    Layout L;
    return make_layout(p, L) ? L.total : 0;
}

lbm_status lbm_init(lbm_sim **out, const lbm_params *p, const uint8_t *solid, const double *rho_init,
                    const double *ux_init, const double *uy_init, void *dev_ws, size_t ws_bytes,
                    void *stream) {
    if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    const std::string why = check_params(p);
    if (!why.empty()) return fail(nullptr, LBM_EINVAL, "%s", why.c_str());
    if (!solid || !rho_init) return fail(nullptr, LBM_EINVAL, "solid and rho_init must not be NULL");
    Layout L;
    if (!make_layout(p, L))
        return fail(nullptr, LBM_EINVAL, "lattice %dx%d too large for one population buffer", p->nx, p->ny);
    if (!dev_ws) return fail(nullptr, LBM_EINVAL, "workspace is NULL");
    if ((uintptr_t)dev_ws % kAlign) return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(nullptr, LBM_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    const size_t n = (size_t)p->nx * p->ny;
    size_t nfluid = 0;
    for (size_t i = 0; i < n; ++i) {
        if (solid[i]) continue;
        ++nfluid;
        const double r = rho_init[i];
        const double u = ux_init ? ux_init[i] : 0.0, v = uy_init ? uy_init[i] : 0.0;
        if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(u) || !std::isfinite(v))
            return fail(nullptr, LBM_EINVAL, "initial density must be > 0 and finite on fluid nodes (node %zu)", i);
    }
    if (nfluid == 0) return fail(nullptr, LBM_EINVAL, "the mask has no fluid node");

    lbm_sim *s = new lbm_sim();
    s->p = *p;
    s->g = L.g;
    s->m = make_model(p);
    s->stream = (hipStream_t)stream;
    if (hipGetDevice(&s->device) != hipSuccess ||
        hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
        hipDeviceGetAttribute(&s->max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, s->device) != hipSuccess) {
        delete s;
        return fail(nullptr, LBM_EDEVICE, "cannot query the current HIP device");
    }
    s->static_scratch = static_scratch_on(s->device, s->static_err);
    char *ws = (char *)dev_ws;
    s->buf[0] = ws + L.buf_off[0];
    s->buf[1] = ws + L.buf_off[1];
    s->buf_bytes = L.buf_bytes;
    s->flags = (uint16_t *)(ws + L.flags_off);
    s->partials = (double *)(ws + L.part_off);
    s->result = (double *)(ws + L.res_off);
    s->rng = (uint32_t *)(ws + L.rng_off);
    s->rowplain = (uint32_t *)(ws + L.rowplain_off);

    // flags, padded to the row pitch
    std::vector<uint16_t> fl;
    derive_flags(p, solid, fl);
    std::vector<uint16_t> padded((size_t)L.g.plane, (uint16_t)lbm::FL_SOLID);
    for (int y = 0; y < p->ny; ++y)
        std::memcpy(&padded[(size_t)y * L.g.pitch], &fl[(size_t)y * p->nx], sizeof(uint16_t) * p->nx);
    // initial fields as float32 [3][ny][nx]
    std::vector<float> stage(3 * n);
    for (size_t i = 0; i < n; ++i) {
        stage[i] = solid[i] ? 0.f : (float)rho_init[i];
        stage[n + i] = (solid[i] || !ux_init) ? 0.f : (float)ux_init[i];
        stage[2 * n + i] = (solid[i] || !uy_init) ? 0.f : (float)uy_init[i];
    }
    auto cleanup = [&](lbm_status st) {
        g_init_error = s->err;
        delete s;
        return st;
    };
    lbm_status st;
#define INIT_TRY(expr)                                                               \
    do {                                                                             \
        hipError_t e_ = (expr);                                                      \
        if (e_ != hipSuccess) {                                                      \
            st = fail(s, LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
            return cleanup(st);                                                      \
        }                                                                            \
    } while (0)
    INIT_TRY(hipMemcpyAsync(s->flags, padded.data(), padded.size() * sizeof(uint16_t),
                            hipMemcpyHostToDevice, s->stream));
    std::vector<uint32_t> plain_rows;
    lbm::row_plain_mask(p->nx, p->ny, fl, plain_rows);
    INIT_TRY(hipMemcpyAsync(s->rowplain, plain_rows.data(), plain_rows.size() * sizeof(uint32_t),
                            hipMemcpyHostToDevice, s->stream));
    INIT_TRY(lbm::launch_fill(s->buf[0], s->buf_bytes, s->stream));
    float *dstage = (float *)s->buf[1];
    INIT_TRY(hipMemcpyAsync(dstage, stage.data(), stage.size() * sizeof(float), hipMemcpyHostToDevice,
                            s->stream));
    INIT_TRY(lbm::launch_init(p->storage, s->buf[0], s->flags, s->g, s->m.rho_off, dstage, dstage + n,
                              dstage + 2 * n, p->nx, s->stream));
    INIT_TRY(lbm::launch_fill(s->buf[1], s->buf_bytes, s->stream));
    INIT_TRY(hipMemcpyAsync(s->rng, s->rng_host, sizeof s->rng_host, hipMemcpyHostToDevice, s->stream));
    INIT_TRY(hipStreamSynchronize(s->stream));
#undef INIT_TRY
    s->cur = 0;
    s->steps = 0;
    *out = s;
    return LBM_OK;
}

lbm_status lbm_init_device(lbm_sim *s, const float *rho, const float *ux, const float *uy) {
    lbm_status st = usable(s);
    if (st) return st;
    if (!rho) return fail(s, LBM_EINVAL, "rho must not be NULL");
    DeviceGuard dg(s->device);
    HIP_TRY(s, lbm::launch_fill(s->buf[s->cur], s->buf_bytes, s->stream));
    HIP_TRY(s, lbm::launch_init(s->p.storage, s->buf[s->cur], s->flags, s->g, s->m.rho_off, rho, ux, uy,
                                s->p.nx, s->stream));
    return LBM_OK;
}

namespace {
// Time steps one launch of a kernel advances (2 or 3 for the multi-step kernels).
int steps_per_launch(int kernel) {
    return kernel == LBM_KERNEL_TWO ? 2 : kernel == LBM_KERNEL_THREE ? 3 : 1;
}

// Columns of one strip (one workgroup's output width) for a kernel.
int strip_columns(const lbm_sim *s, int kernel) {
    switch (kernel) {
    case LBM_KERNEL_WIDE2: return 2 * s->block_x;
    case LBM_KERNEL_WIDE4: return 4 * s->block_x;
    case LBM_KERNEL_TWO:
    case LBM_KERNEL_THREE: return s->block_x - 2 * (2 * steps_per_launch(kernel) - 1);
    default: return s->block_x;
    }
}

// Launch arguments of a step kernel for the handle's current tile; `cache`
// holds that kernel's row chunking (0 = recompute).
lbm::StepArgs step_args_for(lbm_sim *s, int kernel, int &cache) {
    const int cols = strip_columns(s, kernel);
    if (cache == 0) {
        const int strips = (s->p.nx + cols - 1) / cols;
        int chunks;
        if (s->rows > 0) {
            chunks = (s->p.ny + s->rows - 1) / s->rows;
        } else {
            // one wave of resident workgroups, chunks of at least 8 rows
            int per_cu;
            switch (kernel) {
            case LBM_KERNEL_TWO:
            case LBM_KERNEL_THREE:
                per_cu = lbm::stepk_blocks_per_cu(s->p.storage, s->block_x, steps_per_launch(kernel), s->m.trt != 0,
                                                  s->m.sround != 0);
                break;
            case LBM_KERNEL_SPLIT: per_cu = lbm::split_blocks_per_cu(s->p.storage, s->block_x); break;
            case LBM_KERNEL_WIDE2: per_cu = lbm::wide_blocks_per_cu(s->p.storage, s->block_x, 2); break;
            case LBM_KERNEL_WIDE4: per_cu = lbm::wide_blocks_per_cu(s->p.storage, s->block_x, 4); break;
            case LBM_KERNEL_FUSED8: per_cu = lbm::step8_blocks_per_cu(s->p.storage, s->block_x, s->m.trt != 0, s->m.sround != 0); break;
            default: per_cu = lbm::step_blocks_per_cu(s->p.storage, s->block_x, s->m.trt != 0, s->m.sround != 0); break;
            }
            const int cap = s->cus * per_cu;
            chunks = std::max(1, cap / strips);
            chunks = std::min(chunks, std::max(1, s->p.ny / 8));
        }
        cache = std::max(1, std::min(chunks, s->p.ny));
    }
    lbm::StepArgs a;
    a.flags = s->flags;
    a.rowplain = s->rowplain;
    a.g = s->g;
    a.m = s->m;
    a.chunks = cache;
    a.ntiles = ((s->p.nx + cols - 1) / cols) * cache;
    a.tiles_per_xcd = (a.ntiles + 7) / 8;
    a.src = s->buf[s->cur];
    a.dst = s->buf[s->cur ^ 1];
    a.rng = s->rng;
    a.par = s->cur;
    a.acc = s->acc;
    return a;
}

lbm::StepArgs step_args(lbm_sim *s) { return step_args_for(s, s->kernel, s->chunks); }

hipError_t launch_on(const lbm_sim *s, const lbm::StepArgs &a, hipStream_t st) {
    switch (s->kernel) {
    case LBM_KERNEL_TWO:
    case LBM_KERNEL_THREE: return lbm::launch_stepk(s->p.storage, a, s->block_x, steps_per_launch(s->kernel), st);
    case LBM_KERNEL_SPLIT: return lbm::launch_step_split(s->p.storage, a, s->block_x, st);
    case LBM_KERNEL_WIDE2: return lbm::launch_step_wide(s->p.storage, a, s->block_x, 2, st);
    case LBM_KERNEL_WIDE4: return lbm::launch_step_wide(s->p.storage, a, s->block_x, 4, st);
    case LBM_KERNEL_FUSED8: return lbm::launch_step8(s->p.storage, a, s->block_x, st);
    default: return lbm::launch_step(s->p.storage, a, s->block_x, st);
    }
}

hipError_t launch(const lbm_sim *s, const lbm::StepArgs &a) { return launch_on(s, a, s->stream); }

// Graphs bake in the tile, kernel and model: any change drops them.
void drop_graphs(lbm_sim *s) {
    for (int k = 0; k < 2; ++k) {
        if (s->gexec[k]) (void)hipGraphExecDestroy(s->gexec[k]);
        if (s->graph[k]) (void)hipGraphDestroy(s->graph[k]);
        s->gexec[k] = nullptr;
        s->graph[k] = nullptr;
    }
}

// A multi-step kernel's LDS at this block_x fits one workgroup on the device.
bool multi_fits(const lbm_sim *s, int kernel, int block_x) {
    return lbm::stepk_lds_bytes(s->p.storage, block_x, steps_per_launch(kernel)) <= (size_t)s->max_lds;
}

// Issue the launches of nsteps steps from buffer parity `par` on stream st:
// launches of the handle's kernel, then the nsteps mod k steps a multi-step
// kernel leaves as fused-kernel launches at the same block_x.  par follows
// the buffer parity (one flip per launch).
hipError_t issue_steps(lbm_sim *s, hipStream_t st, int64_t nsteps, int &par) {
    const int k = steps_per_launch(s->kernel);
    lbm::StepArgs a = step_args(s);
    for (int64_t n = 0; n + k <= nsteps; n += k) {
        a.src = s->buf[par];
        a.dst = s->buf[par ^ 1];
        a.par = par;
        const hipError_t e = launch_on(s, a, st);
        if (e != hipSuccess) return e;
        par ^= 1;
    }
    const int rem = (int)(nsteps % k);
    if (rem) {
        lbm::StepArgs b = step_args_for(s, LBM_KERNEL_FUSED, s->chunks1);
        for (int r = 0; r < rem; ++r) {
            b.src = s->buf[par];
            b.dst = s->buf[par ^ 1];
            b.par = par;
            const hipError_t e = lbm::launch_step(s->p.storage, b, s->block_x, st);
            if (e != hipSuccess) return e;
            par ^= 1;
        }
    }
    return hipSuccess;
}

// Launches of nsteps steps (see issue_steps).
int64_t launches_for(const lbm_sim *s, int64_t nsteps) {
    const int k = steps_per_launch(s->kernel);
    return nsteps / k + nsteps % k;
}

// Capture the launches of graph_steps steps starting from buffer `parity` on the private
// stream (kernel launches only: no memset or copy nodes).
lbm_status capture_graph(lbm_sim *s, int parity) {
    if (!s->cap && hipStreamCreateWithFlags(&s->cap, hipStreamNonBlocking) != hipSuccess) {
        s->cap = nullptr;
        return fail(s, LBM_EDEVICE, "cannot create the capture stream");
    }
    HIP_TRY(s, hipStreamBeginCapture(s->cap, hipStreamCaptureModeRelaxed));
    int par = parity;
    const hipError_t e = issue_steps(s, s->cap, s->graph_steps, par);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(s->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(s, LBM_EDEVICE, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(s, LBM_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
    }
    s->graph[parity] = g;
    s->gexec[parity] = x;
    return LBM_OK;
}
}  // namespace

lbm_status lbm_step(lbm_sim *s, int64_t nsteps) {
    lbm_status st = usable(s);
    if (st) return st;
    if (nsteps < 0) return fail(s, LBM_EINVAL, "nsteps must be >= 0");
    DeviceGuard dg(s->device);
    int64_t left = nsteps;
    if (s->graph_steps > 0) {
        while (left >= s->graph_steps) {
            if (!s->gexec[s->cur] && (st = capture_graph(s, s->cur)) != LBM_OK) return st;
            HIP_TRY(s, hipGraphLaunch(s->gexec[s->cur], s->stream));
            left -= s->graph_steps;
            s->steps += s->graph_steps;
            if (launches_for(s, s->graph_steps) & 1) s->cur ^= 1;     // each launch flips the buffer parity
        }
    }
    int par = s->cur;
    HIP_TRY(s, issue_steps(s, s->stream, left, par));
    s->cur = par;
    s->steps += left;
    return LBM_OK;
}

lbm_status lbm_profile(lbm_sim *s, double *ux_mean) {
    lbm_status st = usable(s);
    if (st) return st;
    if (!ux_mean) return fail(s, LBM_EINVAL, "ux_mean must not be NULL");
    DeviceGuard dg(s->device);
    double *d = (double *)s->buf[s->cur ^ 1];     // staged in the spare population buffer
    HIP_TRY(s, lbm::launch_profile(s->p.storage, s->buf[s->cur], s->flags, s->g, s->m.rho_off, d, s->stream));
    HIP_TRY(s, hipMemcpyAsync(ux_mean, d, sizeof(double) * (size_t)s->p.ny, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_moments(lbm_sim *s, float *rho, float *ux, float *uy, int on_device) {
    lbm_status st = usable(s);
    if (st) return st;
    DeviceGuard dg(s->device);
    const size_t n = (size_t)s->p.nx * s->p.ny;
    if (on_device) {
        HIP_TRY(s, lbm::launch_moments(s->p.storage, s->buf[s->cur], s->flags, s->g, s->m.rho_off, rho, ux,
                                       uy, s->stream));
        return LBM_OK;
    }
    // stage in the spare population buffer, then copy out
    float *d = (float *)s->buf[s->cur ^ 1];
    HIP_TRY(s, lbm::launch_moments(s->p.storage, s->buf[s->cur], s->flags, s->g, s->m.rho_off,
                                   rho ? d : nullptr, ux ? d + n : nullptr, uy ? d + 2 * n : nullptr,
                                   s->stream));
    if (rho) HIP_TRY(s, hipMemcpyAsync(rho, d, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    if (ux) HIP_TRY(s, hipMemcpyAsync(ux, d + n, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    if (uy) HIP_TRY(s, hipMemcpyAsync(uy, d + 2 * n, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_flux(lbm_sim *s, double *Q, double *M) {
    lbm_status st = usable(s);
    if (st) return st;
    DeviceGuard dg(s->device);
    return do_flux(s, Q, M, s->partials, s->result);
}

lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, int32_t per_lane, void *stream) {
    if (!dst || !src) return fail(nullptr, LBM_EINVAL, "lbm_stream_copy: NULL pointer");
    if (bytes % 16 || (uintptr_t)dst % 16 || (uintptr_t)src % 16)
        return fail(nullptr, LBM_EINVAL, "lbm_stream_copy: pointers and size must be multiples of 16 bytes");
    if (per_lane != 1 && per_lane != 2 && per_lane != 4)
        return fail(nullptr, LBM_EINVAL, "lbm_stream_copy: per_lane must be 1, 2 or 4");
    const char *d = (const char *)dst, *sr = (const char *)src;
    if (d < sr + bytes && sr < d + bytes) return fail(nullptr, LBM_EINVAL, "lbm_stream_copy: buffers overlap");
    const hipError_t e = lbm::launch_stream_copy(dst, src, bytes, per_lane, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, "lbm_stream_copy: %s", hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_round_sr(const float *in, const uint32_t *r, uint16_t *out, int64_t n, int32_t storage,
                        void *stream) {
    if (n < 0 || n > 0xFFFFFFFFll) return fail(nullptr, LBM_EINVAL, "lbm_round_sr: n must be in [0, 2^32)");
    if (storage != LBM_F16 && storage != LBM_BF16)
        return fail(nullptr, LBM_EINVAL, "lbm_round_sr: storage must be LBM_F16 or LBM_BF16");
    if (n > 0 && (!in || !r || !out)) return fail(nullptr, LBM_EINVAL, "lbm_round_sr: NULL pointer");
    const hipError_t e = lbm::launch_round_sr(in, r, out, (uint32_t)n, storage, (hipStream_t)stream);
    if (e != hipSuccess) return fail(nullptr, LBM_EDEVICE, "lbm_round_sr: %s", hipGetErrorString(e));
    return LBM_OK;
}

lbm_status lbm_flux_static(lbm_sim *s, double *Q, double *M) {
    lbm_status st = usable(s);
    if (st) return st;
    if (!s->static_scratch) return fail(s, LBM_EDEVICE, "no static scratch on device %d: %s", s->device,
                                        s->static_err.c_str());
    if ((size_t)lbm::reduce_blocks(s->g) * 4 > kStaticPartials)
        return fail(s, LBM_EINVAL, "lbm_flux_static: %d reduction workgroups exceed the static scratch (%zu)",
                    lbm::reduce_blocks(s->g), kStaticPartials / 4);
    DeviceGuard dg(s->device);
    // k_reduce writes every partial it uses and k_reduce_final the whole
    // result, so nothing needs clearing between calls
    return do_flux(s, Q, M, s->static_scratch, s->static_scratch + kStaticPartials);
}

lbm_status lbm_geometry(lbm_sim *s, uint16_t *flags) {
    lbm_status st = usable(s);
    if (st) return st;
    if (!flags) return fail(s, LBM_EINVAL, "flags must not be NULL");
    DeviceGuard dg(s->device);
    HIP_TRY(s, hipMemcpy2DAsync(flags, (size_t)s->p.nx * sizeof(uint16_t), s->flags,
                                (size_t)s->g.pitch * sizeof(uint16_t), (size_t)s->p.nx * sizeof(uint16_t),
                                (size_t)s->p.ny, hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_set_forces(lbm_sim *s, double f_elec, double accel_x, double accel_y) {
    lbm_status st = usable(s);
    if (st) return st;
    if (!std::isfinite(f_elec) || !std::isfinite(accel_x) || !std::isfinite(accel_y))
        return fail(s, LBM_EINVAL, "forces must be finite");
    s->p.f_elec = f_elec;
    s->p.accel_x = accel_x;
    s->p.accel_y = accel_y;
    s->m = make_model(&s->p);
    drop_graphs(s);
    return LBM_OK;
}

lbm_status lbm_set_tile(lbm_sim *s, int32_t block_x, int32_t rows) {
    lbm_status st = usable(s);
    if (st) return st;
    if (block_x != 64 && block_x != 128 && block_x != 256 && block_x != 512)
        return fail(s, LBM_EINVAL, "block_x must be 64, 128, 256 or 512");
    if (s->kernel == LBM_KERNEL_SPLIT && block_x != 128 && block_x != 256)
        return fail(s, LBM_EINVAL, "the split kernel takes block_x 128 or 256");
    if ((s->kernel == LBM_KERNEL_WIDE2 || s->kernel == LBM_KERNEL_WIDE4) && block_x > 256)
        return fail(s, LBM_EINVAL, "the wide kernels take block_x 64, 128 or 256");
    if (steps_per_launch(s->kernel) > 1 && block_x < 256)
        return fail(s, LBM_EINVAL, "the multi-step kernels take block_x 256 or 512");
    if (steps_per_launch(s->kernel) > 1 && !multi_fits(s, s->kernel, block_x))
        return fail(s, LBM_EINVAL, "the %d-step kernel at block_x %d needs %zu bytes of LDS per workgroup (device: %d)",
                    steps_per_launch(s->kernel), block_x,
                    lbm::stepk_lds_bytes(s->p.storage, block_x, steps_per_launch(s->kernel)), s->max_lds);
    if (rows < 0) return fail(s, LBM_EINVAL, "rows_per_block must be >= 0");
    s->block_x = block_x;
    s->rows = rows;
    s->chunks = 0;
    s->chunks1 = 0;
    drop_graphs(s);
    return LBM_OK;
}

lbm_status lbm_set_accel_field(lbm_sim *s, const float *acc) {
    lbm_status st = usable(s);
    if (st) return st;
    if (acc) {
        if (s->m.trt || s->m.sround)
            return fail(s, LBM_EINVAL, "an acceleration field runs with LBM_COLLIDE_BGK and nearest rounding only");
        if (s->kernel != LBM_KERNEL_FUSED)
            return fail(s, LBM_EINVAL, "an acceleration field runs in LBM_KERNEL_FUSED only");
    }
    s->acc = acc;
    drop_graphs(s);
    return LBM_OK;
}

lbm_status lbm_set_kernel(lbm_sim *s, int32_t kernel) {
    lbm_status st = usable(s);
    if (st) return st;
    if (kernel < LBM_KERNEL_FUSED || kernel > LBM_KERNEL_THREE)
        return fail(s, LBM_EINVAL, "kernel must be one of LBM_KERNEL_FUSED, _SPLIT, _WIDE2, _WIDE4, _FUSED8, _TWO, _THREE");
    const bool trt_sr_ok = kernel == LBM_KERNEL_FUSED || kernel == LBM_KERNEL_FUSED8 || steps_per_launch(kernel) > 1;
    if (s->m.trt && !trt_sr_ok)
        return fail(s, LBM_EINVAL, "the TRT operator runs in LBM_KERNEL_FUSED, _FUSED8, _TWO and _THREE only");
    if (s->m.sround && !trt_sr_ok)
        return fail(s, LBM_EINVAL, "stochastic rounding runs in LBM_KERNEL_FUSED, _FUSED8, _TWO and _THREE only");
    if (s->acc && kernel != LBM_KERNEL_FUSED)
        return fail(s, LBM_EINVAL, "an acceleration field runs in LBM_KERNEL_FUSED only");
    s->kernel = kernel;
    if (kernel == LBM_KERNEL_SPLIT && s->block_x != 128 && s->block_x != 256) s->block_x = 128;
    if ((kernel == LBM_KERNEL_WIDE2 || kernel == LBM_KERNEL_WIDE4) && s->block_x > 256) s->block_x = 256;
    if (steps_per_launch(kernel) > 1 && s->block_x < 256) s->block_x = 256;
    if (steps_per_launch(kernel) > 1 && !multi_fits(s, kernel, s->block_x)) s->block_x = 256;
    s->chunks = 0;
    s->chunks1 = 0;
    drop_graphs(s);
    return LBM_OK;
}

lbm_status lbm_set_graph(lbm_sim *s, int32_t steps_per_graph) {
    lbm_status st = usable(s);
    if (st) return st;
    if (steps_per_graph != 0 && (steps_per_graph < 2 || steps_per_graph > 4096 || steps_per_graph % 2))
        return fail(s, LBM_EINVAL, "steps_per_graph must be 0 or an even number in [2, 4096]");
    DeviceGuard dg(s->device);
    drop_graphs(s);
    s->graph_steps = steps_per_graph;
    return LBM_OK;
}

lbm_status lbm_get_tile(const lbm_sim *s, int32_t *kernel, int32_t *block_x, int32_t *rows) {
    if (!s) return LBM_EINVAL;
    if (kernel) *kernel = s->kernel;
    if (block_x) *block_x = s->block_x;
    if (rows) *rows = s->rows;
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_sim *s, int32_t reps, int32_t *block_x, int32_t *rows, float *us_per_step) {
    lbm_status st = usable(s);
    if (st) return st;
    if (s->acc) return fail(s, LBM_EINVAL, "lbm_autotune: clear the acceleration field first");
    if (reps < 1) return fail(s, LBM_EINVAL, "reps must be >= 1");
    DeviceGuard dg(s->device);
    struct Cand { int kernel, bx; };
    static const Cand kCand[] = {{LBM_KERNEL_FUSED, 64},  {LBM_KERNEL_FUSED, 128}, {LBM_KERNEL_FUSED, 256},
                                 {LBM_KERNEL_FUSED, 512}, {LBM_KERNEL_WIDE2, 64},  {LBM_KERNEL_WIDE2, 128},
                                 {LBM_KERNEL_WIDE2, 256}, {LBM_KERNEL_WIDE4, 64},  {LBM_KERNEL_WIDE4, 128},
                                 {LBM_KERNEL_SPLIT, 128}, {LBM_KERNEL_SPLIT, 256}, {LBM_KERNEL_FUSED8, 128},
                                 {LBM_KERNEL_FUSED8, 256}, {LBM_KERNEL_FUSED8, 512}, {LBM_KERNEL_TWO, 256},
                                 {LBM_KERNEL_TWO, 512},    {LBM_KERNEL_THREE, 256},  {LBM_KERNEL_THREE, 512}};
    static const int kRows[] = {0, 4, 8, 16, 32, 64, 128};
    hipEvent_t e0, e1;
    HIP_TRY(s, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(s, LBM_EDEVICE, "hipEventCreate failed");
    }
    const int keep_bx = s->block_x, keep_rows = s->rows, keep_kernel = s->kernel;
    float best = 0.f;
    int best_bx = keep_bx, best_rows = keep_rows, best_kernel = keep_kernel;
    lbm_status res = LBM_OK;
    for (const Cand &cand : kCand) {
        const int bx = cand.bx;
        const int kst = steps_per_launch(cand.kernel);
        if ((s->m.trt || s->m.sround) && cand.kernel != LBM_KERNEL_FUSED && cand.kernel != LBM_KERNEL_FUSED8 && kst == 1)
            continue;
        if (kst > 1 && !multi_fits(s, cand.kernel, bx)) continue;
        // the multi-step kernels recompute 2 (2k - 1) halo rows per chunk, so they
        // are also tried at the chunk heights that give exactly j resident
        // workgroups per compute unit (j = 1 .. their occupancy): longer chunks
        // against more waves
        std::vector<int> rows_list(std::begin(kRows), std::end(kRows));
        if (kst > 1) {
            const int cols = bx - 2 * (2 * kst - 1);
            const int strips = (s->p.nx + cols - 1) / cols;
            const int per_cu = lbm::stepk_blocks_per_cu(s->p.storage, bx, kst, s->m.trt != 0, s->m.sround != 0);
            for (int k = 1; k <= per_cu; ++k) {
                const int chunks = std::max(1, (k * s->cus) / strips);
                const int r = (s->p.ny + chunks - 1) / chunks;
                if (std::find(rows_list.begin(), rows_list.end(), r) == rows_list.end()) rows_list.push_back(r);
            }
        }
        for (int r : rows_list) {
            if (r > 0 && r >= s->p.ny) continue;
            s->kernel = cand.kernel;
            s->block_x = bx;
            s->rows = r;
            s->chunks = 0;
            s->chunks1 = 0;
            // trial launches read the current buffer and write the spare one,
            // so the state is left as it was
            lbm::StepArgs a = step_args(s);
            hipError_t e = launch(s, a);
            if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
            for (int k = 0; k < reps && e == hipSuccess; ++k) e = launch(s, a);
            if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                res = fail(s, LBM_EDEVICE, "autotune trial %dx%d failed: %s", bx, r, hipGetErrorString(e));
                break;
            }
            // per step: a launch of a multi-step kernel advances kst
            const float us = 1000.f * ms / (float)reps / (float)kst;
            if (best == 0.f || us < best) {
                best = us;
                best_bx = bx;
                best_rows = r;
                best_kernel = cand.kernel;
            }
        }
        if (res != LBM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graphs(s);
    if (res != LBM_OK) {
        s->kernel = keep_kernel;
        s->block_x = keep_bx;
        s->rows = keep_rows;
        s->chunks = 0;
        s->chunks1 = 0;
        return res;
    }
    s->kernel = best_kernel;
    s->block_x = best_bx;
    s->rows = best_rows;
    s->chunks = 0;
    s->chunks1 = 0;
    if (block_x) *block_x = best_bx;
    if (rows) *rows = best_rows;
    if (us_per_step) *us_per_step = best;
    return LBM_OK;
}

size_t lbm_state_bytes(const lbm_sim *s) {
    if (!s) return 0;
    return 2 * sizeof(uint64_t) + (size_t)9 * s->g.plane * elem_size(s->p.storage);
}

lbm_status lbm_save_state(lbm_sim *s, void *host, size_t bytes) {
    lbm_status st = usable(s);
    if (st) return st;
    if (!host || bytes < lbm_state_bytes(s)) return fail(s, LBM_EINVAL, "host buffer too small");
    DeviceGuard dg(s->device);
    uint64_t hdr[2] = {kStateMagic, (uint64_t)s->steps};
    std::memcpy(host, hdr, sizeof hdr);
    HIP_TRY(s, hipMemcpyAsync((char *)host + sizeof hdr, s->buf[s->cur], lbm_state_bytes(s) - sizeof hdr,
                              hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    return LBM_OK;
}

lbm_status lbm_load_state(lbm_sim *s, const void *host, size_t bytes) {
    lbm_status st = usable(s);
    if (st) return st;
    if (!host || bytes < lbm_state_bytes(s)) return fail(s, LBM_EINVAL, "host buffer too small");
    uint64_t hdr[2];
    std::memcpy(hdr, host, sizeof hdr);
    if (hdr[0] != kStateMagic) return fail(s, LBM_EINVAL, "not an lbm state buffer");
    DeviceGuard dg(s->device);
    HIP_TRY(s, hipMemcpyAsync(s->buf[s->cur], (const char *)host + sizeof hdr, lbm_state_bytes(s) - sizeof hdr,
                              hipMemcpyHostToDevice, s->stream));
    // the stochastic-rounding count of the next step is the state's step number
    s->rng_host[s->cur] = (uint32_t)hdr[1];
    HIP_TRY(s, hipMemcpyAsync(s->rng + s->cur, s->rng_host + s->cur, sizeof(uint32_t), hipMemcpyHostToDevice,
                              s->stream));
    HIP_TRY(s, hipStreamSynchronize(s->stream));
    s->steps = (int64_t)hdr[1];
    return LBM_OK;
}

int64_t lbm_steps_done(const lbm_sim *s) { return s ? s->steps : -1; }

void lbm_free(lbm_sim *s) {
    if (!s) return;
    {
        DeviceGuard dg(s->device);
        drop_graphs(s);
        if (s->cap) (void)hipStreamDestroy(s->cap);
    }
    delete s;
}

const char *lbm_last_error(const lbm_sim *s) {
    if (!s) return g_init_error.c_str();
    return s->err.c_str();
}

const char *lbm_status_string(int st) {
    switch (st) {
    case LBM_OK: return "LBM_OK";
    case LBM_EINVAL: return "LBM_EINVAL";
    case LBM_ENOMEM: return "LBM_ENOMEM";
    case LBM_EDEVICE: return "LBM_EDEVICE";
    case LBM_EDIVERGED: return "LBM_EDIVERGED";
    case LBM_ESTATE: return "LBM_ESTATE";
    default: return "unknown lbm_status";
    }
}

}  // extern "C"
