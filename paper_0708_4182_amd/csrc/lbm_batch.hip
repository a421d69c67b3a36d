// Host side of the batched engine: many independent lattices ("channels") of
// uneven sizes advanced together by one kernel launch per time step (a
// persistent grid fed by a tile queue, or one workgroup per tile), optionally
// replayed as a hipGraph of K steps.  Declared in
// include/lbm.h (lbm_batch_*).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"

using lbm::ChannelDesc;
using lbm::Grid;
using lbm::Model;

namespace lbm {
// shared with lbm_api.hip
std::string check_params_str(const lbm_params *p);
Model make_model_of(const lbm_params *p);
float storage_offset_of(const lbm_params *p);
void derive_flags_of(const lbm_params *p, const uint8_t *solid, std::vector<uint16_t> &out);
void row_plain_mask(int nx, int ny, const std::vector<uint16_t> &fl, std::vector<uint32_t> &mask);
}  // namespace lbm

namespace {
constexpr size_t kAlign = 256;
constexpr int kMaxGraphSteps = 1024;
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
size_t elem_size(int storage) { return storage == LBM_F32 ? 4 : 2; }
thread_local std::string g_batch_init_error;

struct BatchLayout {
    std::vector<Grid> g;
    std::vector<size_t> buf0, buf1, flags, rowplain;
    size_t buf_bytes_max = 0;
    size_t descs, tiles, tiles_k, counters, ids, cur, out, rng, total;
    size_t max_tiles;
};

// Largest possible tile count: strips of 64 columns, chunks of at least 8 rows.
size_t tile_bound(const lbm_params &p) {
    return (size_t)((p.nx + 63) / 64) * (size_t)(p.ny / 8 + 1);
}

bool make_batch_layout(int n, const lbm_params *p, BatchLayout &L, std::string &why) {
    if (n <= 0 || n > 65535) {
        why = "n must be in [1, 65535]";
        return false;
    }
    size_t off = 0;
    L.max_tiles = 0;
    for (int i = 0; i < n; ++i) {
        const std::string w = lbm::check_params_str(&p[i]);
        if (!w.empty()) {
            why = "channel " + std::to_string(i) + ": " + w;
            return false;
        }
        if (p[i].collision != p[0].collision) {
            why = "all channels must use the same collision operator";
            return false;
        }
        if (p[i].rounding != p[0].rounding) {
            why = "all channels must use the same rounding";
            return false;
        }
        if (p[i].storage != p[0].storage) {
            why = "all channels must use the same storage";
            return false;
        }
        Grid g;
        g.nx = p[i].nx;
        g.ny = p[i].ny;
        g.pitch = (int32_t)align_up((size_t)p[i].nx, 64);
        const size_t plane = (size_t)g.pitch * g.ny;
        const size_t bytes = 9 * plane * elem_size(p[i].storage);
        if (bytes >= (size_t(1) << 32) || 3 * (size_t)p[i].nx * p[i].ny * 4 > align_up(bytes, kAlign)) {
            why = "channel " + std::to_string(i) + " too large";
            return false;
        }
        if (tile_bound(p[i]) > 65535) {
            why = "channel " + std::to_string(i) + " has too many tiles";
            return false;
        }
        g.plane = (uint32_t)plane;
        L.g.push_back(g);
        L.buf0.push_back(off);
        off += align_up(bytes, kAlign);
        L.buf1.push_back(off);
        off += align_up(bytes, kAlign);
        L.flags.push_back(off);
        off += align_up(plane * 2, kAlign);
        L.rowplain.push_back(off);
        off += align_up(4 * (size_t)((g.ny + 31) / 32), kAlign);
        L.max_tiles += tile_bound(p[i]);
        L.buf_bytes_max = std::max(L.buf_bytes_max, align_up(bytes, kAlign));
    }
    L.descs = off;
    off += align_up(sizeof(ChannelDesc) * n, kAlign);
    L.tiles = off;
    off += align_up(4 * L.max_tiles, kAlign);
    L.tiles_k = off;                  // the multi-step kernel's list (wider strips: never longer)
    off += align_up(4 * L.max_tiles, kAlign);
    L.counters = off;
    off += align_up(4 * kMaxGraphSteps, kAlign);
    L.ids = off;
    off += align_up(4 * (size_t)n, kAlign);
    L.cur = off;
    off += align_up(4 * (size_t)n, kAlign);
    L.out = off;
    off += align_up(32 * (size_t)n, kAlign);
    L.rng = off;
    off += kAlign;
    L.total = off;
    return true;
}
}  // namespace

struct lbm_batch {
    int n = 0;
    int storage = 0;
    bool trt = false;           // collision operator of every channel
    bool sround = false;        // stochastic rounding of every channel
    uint32_t *d_rng = nullptr;  // two-slot step counter of stochastic rounding
    uint32_t rng_host[2] = {0u, 0u};
    std::vector<lbm_params> p;
    std::vector<Grid> g;
    std::vector<ChannelDesc> desc;     // host mirror of the device table
    std::vector<char *> buf0, buf1;
    std::vector<uint16_t *> flags;
    std::vector<uint32_t *> rowplain;
    ChannelDesc *d_desc = nullptr;
    uint32_t *d_tiles = nullptr;
    uint32_t *d_tiles_k = nullptr;     // tiles of the multi-step kernel
    uint32_t *d_counters = nullptr;
    int32_t *d_ids = nullptr, *d_cur = nullptr;
    double *d_out = nullptr;
    size_t max_tiles = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap = nullptr;         // private stream used only for graph capture
    int device = 0, cus = 0;
    std::vector<uint8_t> active;
    std::vector<int32_t> cur;          // current buffer index per channel
    std::vector<int64_t> steps;
    int parity = 0;                    // current buffer index of the active channels
    int block_x = 256;
    int tile_rows = 32;
    int ntiles = 0;
    int kstep = 1;                     // time steps per launch: 1, or 2 / 3 (k_batch_tilesk)
    int kbx = 256;                     // block_x of the multi-step kernel (256 or 512)
    int ntiles_k = 0;
    bool tiles_dirty = true;
    std::vector<uint32_t> host_tiles, host_tiles_k;
    std::vector<int32_t> host_ids;
    int graph_steps = 0;
    int persistent = 0;                // 1: persistent queue kernel, 0: one workgroup per tile
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    lbm_status sticky = LBM_OK;
    std::string err;
};

namespace {

lbm_status bfail(lbm_batch *b, lbm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (b) {
        b->err = buf;
        if (st == LBM_EDEVICE) b->sticky = st;
    } else {
        g_batch_init_error = buf;
    }
    return st;
}

#define BHIP(b, expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return bfail((b), LBM_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));      \
    } while (0)

lbm_status busable(lbm_batch *b) {
    if (!b) return LBM_EINVAL;
    if (b->sticky != LBM_OK) return LBM_ESTATE;
    return LBM_OK;
}

void drop_graphs(lbm_batch *b) {
    for (int k = 0; k < 2; ++k) {
        if (b->gexec[k]) (void)hipGraphExecDestroy(b->gexec[k]);
        if (b->graph[k]) (void)hipGraphDestroy(b->graph[k]);
        b->gexec[k] = nullptr;
        b->graph[k] = nullptr;
    }
}

int chunks_for(int ny, int rows) {
    int c = (ny + rows / 2) / rows;
    c = std::max(1, std::min(c, std::max(1, ny / 8)));
    return c;
}

// Rebuild the tile list of the active channels (largest first) and upload it.
lbm_status upload_tiles(lbm_batch *b) {
    std::vector<int> order;
    for (int i = 0; i < b->n; ++i)
        if (b->active[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (int64_t)b->g[a].nx * b->g[a].ny > (int64_t)b->g[c].nx * b->g[c].ny;
    });
    b->host_tiles.clear();
    b->host_tiles_k.clear();
    const int kcols = b->kbx - 2 * (2 * std::max(b->kstep, 2) - 1);   // output columns of a multi-step strip
    for (int i : order) {
        const int strips = (b->g[i].nx + b->block_x - 1) / b->block_x;
        const int chunks = chunks_for(b->g[i].ny, b->tile_rows);
        b->desc[i].chunks = chunks;
        for (int t = 0; t < strips * chunks; ++t) b->host_tiles.push_back(((uint32_t)i << 16) | (uint32_t)t);
        if (b->kstep > 1) {
            const int kstrips = (b->g[i].nx + kcols - 1) / kcols;
            b->desc[i].chunks_k = chunks;
            for (int t = 0; t < kstrips * chunks; ++t)
                b->host_tiles_k.push_back(((uint32_t)i << 16) | (uint32_t)t);
        }
    }
    if (b->host_tiles.size() > b->max_tiles || b->host_tiles_k.size() > b->max_tiles)
        return bfail(b, LBM_EINVAL, "tile list overflow");
    b->ntiles = (int)b->host_tiles.size();
    b->ntiles_k = (int)b->host_tiles_k.size();
    BHIP(b, hipMemcpyAsync(b->d_desc, b->desc.data(), sizeof(ChannelDesc) * b->n, hipMemcpyHostToDevice,
                           b->stream));
    if (b->ntiles)
        BHIP(b, hipMemcpyAsync(b->d_tiles, b->host_tiles.data(), 4 * b->host_tiles.size(),
                               hipMemcpyHostToDevice, b->stream));
    if (b->ntiles_k)
        BHIP(b, hipMemcpyAsync(b->d_tiles_k, b->host_tiles_k.data(), 4 * b->host_tiles_k.size(),
                               hipMemcpyHostToDevice, b->stream));
    // pageable sources: make sure the copies are done before the vectors change
    BHIP(b, hipStreamSynchronize(b->stream));
    b->tiles_dirty = false;
    drop_graphs(b);
    return LBM_OK;
}

// Grid of a step launch: the persistent grid, or 0 for one workgroup per tile.
int persistent_grid(lbm_batch *b) {
    if (!b->persistent) return 0;
    const int per_cu = lbm::batch_blocks_per_cu(b->storage, b->block_x, b->trt, b->sround);
    return std::max(1, std::min(b->ntiles, b->cus * per_cu));
}

hipError_t enqueue_step(lbm_batch *b, hipStream_t s, int slot, int parity, int grid) {
    lbm::BatchStepArgs a;
    a.descs = b->d_desc;
    a.tiles = b->d_tiles;
    a.counters = b->d_counters;
    a.ntiles = b->ntiles;
    a.slot = slot;
    a.parity = parity;
    a.trt = b->trt ? 1 : 0;
    a.sround = b->sround ? 1 : 0;
    a.rng = b->d_rng;
    return lbm::launch_batch_step(b->storage, a, b->block_x, grid, s);
}

// One launch of the multi-step kernel: kstep time steps from buffer `parity`.
hipError_t enqueue_stepk(lbm_batch *b, hipStream_t s, int parity) {
    lbm::BatchStepArgs a;
    a.descs = b->d_desc;
    a.tiles = b->d_tiles_k;
    a.counters = b->d_counters;
    a.ntiles = b->ntiles_k;
    a.slot = 0;
    a.parity = parity;
    a.trt = b->trt ? 1 : 0;
    a.sround = b->sround ? 1 : 0;
    a.rng = b->d_rng;
    return lbm::launch_batch_stepk(b->storage, a, b->kbx, b->kstep, s);
}

// Launches of nsteps steps: nsteps / kstep multi-step launches, then the rest
// one step each; each launch flips the buffer parity.
int launches_of(const lbm_batch *b, int64_t nsteps) {
    return (int)(nsteps / b->kstep + nsteps % b->kstep);
}

lbm_status capture_graph(lbm_batch *b, int parity) {
    const int K = b->graph_steps, grid = persistent_grid(b);
    BHIP(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
    hipError_t e = grid > 0 ? lbm::launch_fill(b->d_counters, align_up(4 * (size_t)K, 16), b->cap) : hipSuccess;
    int par = parity, slot = 0, left = K;
    for (; b->kstep > 1 && left >= b->kstep && e == hipSuccess; left -= b->kstep, par ^= 1)
        e = enqueue_stepk(b, b->cap, par);
    for (; left > 0 && e == hipSuccess; --left, par ^= 1) e = enqueue_step(b, b->cap, slot++, par, grid);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bfail(b, LBM_EDEVICE, "graph capture failed: %s",
                     hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t x = nullptr;
    const hipError_t e3 = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(g);
        return bfail(b, LBM_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e3));
    }
    b->graph[parity] = g;
    b->gexec[parity] = x;
    return LBM_OK;
}

lbm_status eager_step(lbm_batch *b, int parity, int grid) {
    if (grid > 0) BHIP(b, lbm::launch_fill(b->d_counters, 16, b->stream));
    BHIP(b, enqueue_step(b, b->stream, 0, parity, grid));
    return LBM_OK;
}

lbm_status eager_stepk(lbm_batch *b, int parity) {
    BHIP(b, enqueue_stepk(b, b->stream, parity));
    return LBM_OK;
}

lbm_status check_index(lbm_batch *b, int32_t i) {
    if (i < 0 || i >= b->n) return bfail(b, LBM_EINVAL, "channel index %d out of range", i);
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params *p) {
    if (!p) return 0;
    BatchLayout L;
    std::string why;
    return make_batch_layout(n, p, L, why) ? L.total : 0;
}

lbm_status lbm_batch_init(lbm_batch **out, int32_t n, const lbm_params *p, const uint8_t *const *solid,
                          const double *const *rho_init, const double *const *ux_init,
                          const double *const *uy_init, void *dev_ws, size_t ws_bytes, void *stream) {
    if (!out) return bfail(nullptr, LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p || !solid || !rho_init) return bfail(nullptr, LBM_EINVAL, "params, solid and rho_init must not be NULL");
    BatchLayout L;
    std::string why;
    if (!make_batch_layout(n, p, L, why)) return bfail(nullptr, LBM_EINVAL, "%s", why.c_str());
    if (!dev_ws || (uintptr_t)dev_ws % kAlign) return bfail(nullptr, LBM_EINVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < L.total) return bfail(nullptr, LBM_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    for (int i = 0; i < n; ++i) {
        if (!solid[i] || !rho_init[i]) return bfail(nullptr, LBM_EINVAL, "channel %d: solid and rho_init must not be NULL", i);
        const size_t m = (size_t)p[i].nx * p[i].ny;
        size_t nfluid = 0;
        for (size_t k = 0; k < m; ++k) {
            if (solid[i][k]) continue;
            ++nfluid;
            const double r = rho_init[i][k];
            const double u = (ux_init && ux_init[i]) ? ux_init[i][k] : 0.0;
            const double v = (uy_init && uy_init[i]) ? uy_init[i][k] : 0.0;
            if (!(r > 0.0) || !std::isfinite(r) || !std::isfinite(u) || !std::isfinite(v))
                return bfail(nullptr, LBM_EINVAL, "channel %d: initial density must be > 0 and finite (node %zu)", i, k);
        }
        if (nfluid == 0) return bfail(nullptr, LBM_EINVAL, "channel %d has no fluid node", i);
    }

    lbm_batch *b = new lbm_batch();
    b->n = n;
    b->storage = p[0].storage;
    b->trt = p[0].collision != LBM_COLLIDE_BGK;   // TRT and MRT share the kernels
    b->sround = p[0].rounding == LBM_ROUND_STOCHASTIC;
    b->p.assign(p, p + n);
    b->g = L.g;
    b->stream = (hipStream_t)stream;
    b->max_tiles = L.max_tiles;
    auto cleanup = [&](lbm_status st) {
        g_batch_init_error = b->err.empty() ? g_batch_init_error : b->err;
        if (b->cap) (void)hipStreamDestroy(b->cap);
        delete b;
        return st;
    };
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess) {
        bfail(b, LBM_EDEVICE, "cannot query the current HIP device");
        return cleanup(LBM_EDEVICE);
    }
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        bfail(b, LBM_EDEVICE, "hipStreamCreateWithFlags failed");
        return cleanup(LBM_EDEVICE);
    }
    char *ws = (char *)dev_ws;
    b->d_desc = (ChannelDesc *)(ws + L.descs);
    b->d_tiles = (uint32_t *)(ws + L.tiles);
    b->d_tiles_k = (uint32_t *)(ws + L.tiles_k);
    b->d_counters = (uint32_t *)(ws + L.counters);
    b->d_ids = (int32_t *)(ws + L.ids);
    b->d_cur = (int32_t *)(ws + L.cur);
    b->d_out = (double *)(ws + L.out);
    b->d_rng = (uint32_t *)(ws + L.rng);
    if (hipMemcpyAsync(b->d_rng, b->rng_host, sizeof b->rng_host, hipMemcpyHostToDevice, b->stream) != hipSuccess) {
        bfail(b, LBM_EDEVICE, "cannot set the rounding step counter");
        return cleanup(LBM_EDEVICE);
    }
    b->desc.resize(n);
    b->active.assign(n, 1);
    b->cur.assign(n, 0);
    b->steps.assign(n, 0);
    for (int i = 0; i < n; ++i) {
        b->buf0.push_back(ws + L.buf0[i]);
        b->buf1.push_back(ws + L.buf1[i]);
        b->flags.push_back((uint16_t *)(ws + L.flags[i]));
        b->rowplain.push_back((uint32_t *)(ws + L.rowplain[i]));
        ChannelDesc &d = b->desc[i];
        std::memset(&d, 0, sizeof d);
        d.g = L.g[i];
        d.m = lbm::make_model_of(&p[i]);
        d.chunks = 1;
        d.buf[0] = b->buf0[i];
        d.buf[1] = b->buf1[i];
        d.flags = b->flags[i];
        d.rowplain = b->rowplain[i];
    }
    // geometry and initial populations, one channel at a time (host staging reused)
    std::vector<uint16_t> fl, padded;
    std::vector<uint32_t> plain_rows;
    std::vector<float> stage;
    for (int i = 0; i < n; ++i) {
        const Grid &g = L.g[i];
        const size_t m = (size_t)g.nx * g.ny;
        lbm::derive_flags_of(&p[i], solid[i], fl);
        padded.assign((size_t)g.plane, (uint16_t)lbm::FL_SOLID);
        for (int y = 0; y < g.ny; ++y)
            std::memcpy(&padded[(size_t)y * g.pitch], &fl[(size_t)y * g.nx], 2 * (size_t)g.nx);
        stage.assign(3 * m, 0.f);
        for (size_t k = 0; k < m; ++k) {
            if (solid[i][k]) continue;
            stage[k] = (float)rho_init[i][k];
            stage[m + k] = (ux_init && ux_init[i]) ? (float)ux_init[i][k] : 0.f;
            stage[2 * m + k] = (uy_init && uy_init[i]) ? (float)uy_init[i][k] : 0.f;
        }
        const size_t bb = 9 * (size_t)g.plane * elem_size(b->storage);
        hipError_t e = hipMemcpyAsync(b->flags[i], padded.data(), 2 * padded.size(), hipMemcpyHostToDevice, b->stream);
        lbm::row_plain_mask(g.nx, g.ny, fl, plain_rows);
        if (e == hipSuccess)
            e = hipMemcpyAsync(b->rowplain[i], plain_rows.data(), 4 * plain_rows.size(), hipMemcpyHostToDevice,
                               b->stream);
        if (e == hipSuccess) e = lbm::launch_fill(b->buf0[i], align_up(bb, 16), b->stream);
        float *dstage = (float *)b->buf1[i];
        if (e == hipSuccess)
            e = hipMemcpyAsync(dstage, stage.data(), 4 * stage.size(), hipMemcpyHostToDevice, b->stream);
        if (e == hipSuccess)
            e = lbm::launch_init(b->storage, b->buf0[i], b->flags[i], g, lbm::storage_offset_of(&p[i]), dstage, dstage + m,
                                 dstage + 2 * m, g.nx, b->stream);
        if (e == hipSuccess) e = lbm::launch_fill(b->buf1[i], align_up(bb, 16), b->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(b->stream);   // host staging is reused
        if (e != hipSuccess) {
            bfail(b, LBM_EDEVICE, "init of channel %d failed: %s", i, hipGetErrorString(e));
            return cleanup(LBM_EDEVICE);
        }
    }
    const lbm_status st = upload_tiles(b);
    if (st != LBM_OK) return cleanup(st);
    *out = b;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps) {
    lbm_status st = busable(b);
    if (st) return st;
    if (nsteps < 0) return bfail(b, LBM_EINVAL, "nsteps must be >= 0");
    if (b->tiles_dirty && (st = upload_tiles(b)) != LBM_OK) return st;
    if (b->ntiles == 0 || nsteps == 0) return LBM_OK;
    const int grid = persistent_grid(b);
    int64_t left = nsteps;
    const int K = b->graph_steps;
    if (K > 0) {
        const int flip = launches_of(b, K) & 1;   // parity change of one replay
        while (left >= K) {
            if (!b->gexec[b->parity] && (st = capture_graph(b, b->parity)) != LBM_OK) return st;
            BHIP(b, hipGraphLaunch(b->gexec[b->parity], b->stream));
            b->parity ^= flip;
            left -= K;
        }
    }
    while (b->kstep > 1 && left >= b->kstep) {
        if ((st = eager_stepk(b, b->parity)) != LBM_OK) return st;
        b->parity ^= 1;
        left -= b->kstep;
    }
    while (left > 0) {
        if ((st = eager_step(b, b->parity, grid)) != LBM_OK) return st;
        b->parity ^= 1;
        --left;
    }
    for (int i = 0; i < b->n; ++i)
        if (b->active[i]) {
            b->steps[i] += nsteps;
            b->cur[i] = b->parity;
        }
    return LBM_OK;
}

lbm_status lbm_batch_flux(lbm_batch *b, double *Q, double *M) {
    lbm_status st = busable(b);
    if (st) return st;
    b->host_ids.resize(b->n);
    std::iota(b->host_ids.begin(), b->host_ids.end(), 0);
    BHIP(b, hipMemcpyAsync(b->d_ids, b->host_ids.data(), 4 * (size_t)b->n, hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipMemcpyAsync(b->d_cur, b->cur.data(), 4 * (size_t)b->n, hipMemcpyHostToDevice, b->stream));
    BHIP(b, lbm::launch_batch_reduce(b->storage, b->d_desc, b->d_ids, b->d_cur, b->n, b->d_out, b->stream));
    std::vector<double> host(4 * (size_t)b->n);
    BHIP(b, hipMemcpyAsync(host.data(), b->d_out, 8 * host.size(), hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    int bad = 0;
    for (int i = 0; i < b->n; ++i) {
        const bool ok = host[4 * i + 2] == 0.0;
        bad += !ok;
        if (Q) Q[i] = ok ? host[4 * i] : NAN;
        if (M) M[i] = host[4 * i + 1];
    }
    if (bad) return bfail(b, LBM_EDIVERGED, "%d channel(s) diverged (their Q is NaN)", bad);
    return LBM_OK;
}

lbm_status lbm_batch_moments(lbm_batch *b, int32_t i, float *rho, float *ux, float *uy, int on_device) {
    lbm_status st = busable(b);
    if (st) return st;
    if ((st = check_index(b, i)) != LBM_OK) return st;
    const Grid &g = b->g[i];
    const size_t m = (size_t)g.nx * g.ny;
    const char *src = b->cur[i] ? b->buf1[i] : b->buf0[i];
    const float off = lbm::storage_offset_of(&b->p[i]);
    if (on_device) {
        BHIP(b, lbm::launch_moments(b->storage, src, b->flags[i], g, off, rho, ux, uy, b->stream));
        return LBM_OK;
    }
    float *d = (float *)(b->cur[i] ? b->buf0[i] : b->buf1[i]);
    BHIP(b, lbm::launch_moments(b->storage, src, b->flags[i], g, off, rho ? d : nullptr, ux ? d + m : nullptr,
                                uy ? d + 2 * m : nullptr, b->stream));
    if (rho) BHIP(b, hipMemcpyAsync(rho, d, 4 * m, hipMemcpyDeviceToHost, b->stream));
    if (ux) BHIP(b, hipMemcpyAsync(ux, d + m, 4 * m, hipMemcpyDeviceToHost, b->stream));
    if (uy) BHIP(b, hipMemcpyAsync(uy, d + 2 * m, 4 * m, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status lbm_batch_profile(lbm_batch *b, int32_t i, double *ux_mean) {
    lbm_status st = busable(b);
    if (st) return st;
    if ((st = check_index(b, i)) != LBM_OK) return st;
    if (!ux_mean) return bfail(b, LBM_EINVAL, "ux_mean must not be NULL");
    const Grid &g = b->g[i];
    const char *src = b->cur[i] ? b->buf1[i] : b->buf0[i];
    double *d = (double *)(b->cur[i] ? b->buf0[i] : b->buf1[i]);
    BHIP(b, lbm::launch_profile(b->storage, src, b->flags[i], g, lbm::storage_offset_of(&b->p[i]), d, b->stream));
    BHIP(b, hipMemcpyAsync(ux_mean, d, sizeof(double) * (size_t)g.ny, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status lbm_batch_geometry(lbm_batch *b, int32_t i, uint16_t *flags) {
    lbm_status st = busable(b);
    if (st) return st;
    if ((st = check_index(b, i)) != LBM_OK) return st;
    if (!flags) return bfail(b, LBM_EINVAL, "flags must not be NULL");
    const Grid &g = b->g[i];
    BHIP(b, hipMemcpy2DAsync(flags, 2 * (size_t)g.nx, b->flags[i], 2 * (size_t)g.pitch, 2 * (size_t)g.nx,
                             (size_t)g.ny, hipMemcpyDeviceToHost, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status lbm_batch_init_device(lbm_batch *b, int32_t i, const float *rho, const float *ux, const float *uy) {
    lbm_status st = busable(b);
    if (st) return st;
    if ((st = check_index(b, i)) != LBM_OK) return st;
    if (!rho) return bfail(b, LBM_EINVAL, "rho must not be NULL");
    const Grid &g = b->g[i];
    char *dst = b->cur[i] ? b->buf1[i] : b->buf0[i];
    const size_t bb = 9 * (size_t)g.plane * elem_size(b->storage);
    BHIP(b, lbm::launch_fill(dst, align_up(bb, 16), b->stream));
    BHIP(b, lbm::launch_init(b->storage, dst, b->flags[i], g, lbm::storage_offset_of(&b->p[i]), rho, ux, uy, g.nx, b->stream));
    b->steps[i] = 0;
    return LBM_OK;
}

lbm_status lbm_batch_set_forces(lbm_batch *b, int32_t i, double f_elec, double accel_x, double accel_y) {
    lbm_status st = busable(b);
    if (st) return st;
    if ((st = check_index(b, i)) != LBM_OK) return st;
    if (!std::isfinite(f_elec) || !std::isfinite(accel_x) || !std::isfinite(accel_y))
        return bfail(b, LBM_EINVAL, "forces must be finite");
    b->p[i].f_elec = f_elec;
    b->p[i].accel_x = accel_x;
    b->p[i].accel_y = accel_y;
    b->desc[i].m = lbm::make_model_of(&b->p[i]);
    BHIP(b, hipMemcpyAsync(b->d_desc + i, &b->desc[i], sizeof(ChannelDesc), hipMemcpyHostToDevice, b->stream));
    BHIP(b, hipStreamSynchronize(b->stream));
    return LBM_OK;
}

lbm_status lbm_batch_retire(lbm_batch *b, const uint8_t *done) {
    lbm_status st = busable(b);
    if (st) return st;
    if (!done) return bfail(b, LBM_EINVAL, "done must not be NULL");
    for (int i = 0; i < b->n; ++i)
        if (done[i]) b->active[i] = 0;
    return upload_tiles(b);
}

lbm_status lbm_batch_set_tile(lbm_batch *b, int32_t block_x, int32_t rows) {
    lbm_status st = busable(b);
    if (st) return st;
    if (block_x != 64 && block_x != 128 && block_x != 256 && block_x != 512)
        return bfail(b, LBM_EINVAL, "block_x must be 64, 128, 256 or 512");
    if (rows < 8) return bfail(b, LBM_EINVAL, "rows_per_tile must be >= 8");
    b->block_x = block_x;
    b->kbx = block_x == 512 ? 512 : 256;
    b->tile_rows = rows;
    return upload_tiles(b);
}

lbm_status lbm_batch_set_schedule(lbm_batch *b, int32_t persistent) {
    lbm_status st = busable(b);
    if (st) return st;
    b->persistent = persistent ? 1 : 0;
    drop_graphs(b);
    return LBM_OK;
}

lbm_status lbm_batch_set_kernel(lbm_batch *b, int32_t kernel) {
    lbm_status st = busable(b);
    if (st) return st;
    const int k = kernel == LBM_KERNEL_FUSED ? 1 : kernel == LBM_KERNEL_TWO ? 2 : kernel == LBM_KERNEL_THREE ? 3 : 0;
    if (!k) return bfail(b, LBM_EINVAL, "kernel must be LBM_KERNEL_FUSED, LBM_KERNEL_TWO or LBM_KERNEL_THREE");
    const int kbx = b->block_x == 512 ? 512 : 256;
    if (k > 1) {
        int max_lds = 0;
        BHIP(b, hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device));
        if (lbm::stepk_lds_bytes(b->storage, kbx, k) > (size_t)max_lds)
            return bfail(b, LBM_EINVAL, "the %d-step kernel at block_x %d needs more LDS than the device has", k, kbx);
    }
    b->kstep = k;
    b->kbx = kbx;
    return upload_tiles(b);
}

int32_t lbm_batch_get_kernel(const lbm_batch *b) {
    if (!b) return -1;
    return b->kstep == 1 ? LBM_KERNEL_FUSED : b->kstep == 2 ? LBM_KERNEL_TWO : LBM_KERNEL_THREE;
}

lbm_status lbm_batch_set_graph(lbm_batch *b, int32_t steps_per_graph) {
    lbm_status st = busable(b);
    if (st) return st;
    if (steps_per_graph < 0 || steps_per_graph > kMaxGraphSteps || (steps_per_graph & 1))
        return bfail(b, LBM_EINVAL, "steps_per_graph must be 0 or an even number <= %d", kMaxGraphSteps);
    drop_graphs(b);
    b->graph_steps = steps_per_graph;
    return LBM_OK;
}

lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, int32_t *block_x, int32_t *rows, float *us_per_step) {
    lbm_status st = busable(b);
    if (st) return st;
    if (reps < 1) return bfail(b, LBM_EINVAL, "reps must be >= 1");
    static const int kBX[] = {64, 128, 256, 512};
    static const int kRows[] = {16, 32, 64};
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return bfail(b, LBM_EDEVICE, "hipEventCreate failed");
    }
    // candidates: the one-step kernel (both schedules, every block_x) and the
    // multi-step kernels (one workgroup per tile, block_x 256 or 512, where the
    // device's LDS allows), each at every chunk height; time per step
    struct Cand { int kstep, pers, bx; };
    std::vector<Cand> cands;
    for (int pers = 0; pers < 2; ++pers)
        for (int bx : kBX) cands.push_back({1, pers, bx});
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, b->device) != hipSuccess)
        max_lds = 0;
    for (int k = 2; k <= 3; ++k)
        for (int bx : {256, 512})
            if (lbm::stepk_lds_bytes(b->storage, bx, k) <= (size_t)max_lds) cands.push_back({k, 0, bx});
    float best = 0.f;
    Cand bestc{b->kstep, b->persistent, b->block_x};
    int best_rows = b->tile_rows;
    for (const Cand &c : cands) {
        for (int r : kRows) {
            b->persistent = c.pers;
            b->kstep = c.kstep;
            b->block_x = c.bx;
            b->kbx = c.bx == 512 ? 512 : 256;
            b->tile_rows = r;
            if ((st = upload_tiles(b)) != LBM_OK) break;
            if ((c.kstep > 1 ? b->ntiles_k : b->ntiles) == 0) continue;
            const int grid = c.kstep > 1 ? 0 : persistent_grid(b);
            // trial launches read the current buffers and write the spare ones
            if ((st = c.kstep > 1 ? eager_stepk(b, b->parity) : eager_step(b, b->parity, grid)) != LBM_OK) break;
            hipError_t e = hipEventRecord(e0, b->stream);
            for (int k = 0; k < reps && e == hipSuccess; ++k) {
                if (c.kstep > 1) {
                    e = enqueue_stepk(b, b->stream, b->parity);
                } else {
                    if (grid > 0) e = lbm::launch_fill(b->d_counters, 16, b->stream);
                    if (e == hipSuccess) e = enqueue_step(b, b->stream, 0, b->parity, grid);
                }
            }
            if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = bfail(b, LBM_EDEVICE, "batch autotune trial failed: %s", hipGetErrorString(e));
                break;
            }
            const float us = 1000.f * ms / (float)(reps * c.kstep);
            if (best == 0.f || us < best) {
                best = us;
                bestc = c;
                best_rows = r;
            }
        }
        if (st != LBM_OK) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != LBM_OK) return st;
    b->kstep = bestc.kstep;
    b->persistent = bestc.pers;
    b->block_x = bestc.bx;
    b->kbx = bestc.bx == 512 ? 512 : 256;
    b->tile_rows = best_rows;
    if ((st = upload_tiles(b)) != LBM_OK) return st;
    if (block_x) *block_x = bestc.bx;
    if (rows) *rows = best_rows;
    if (us_per_step) *us_per_step = best;
    return LBM_OK;
}

int64_t lbm_batch_steps_done(const lbm_batch *b, int32_t i) {
    if (!b || i < 0 || i >= b->n) return -1;
    return b->steps[i];
}

void lbm_batch_free(lbm_batch *b) {
    if (!b) return;
    drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
}

const char *lbm_batch_last_error(const lbm_batch *b) {
    if (!b) return g_batch_init_error.c_str();
    return b->err.c_str();
}

}  // extern "C"
