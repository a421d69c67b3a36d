// Sanitizer driver for the host side of liblbm (test infrastructure).  Built
// by tests/test_sanitizers.py together with the library's sources, host code
// only, with -fsanitize=address,undefined, and run on a machine without a GPU:
//   - workspace layouts (lbm_workspace_bytes, lbm_batch_workspace_bytes) for
//     ragged sizes, including ny < 32 and ny not a multiple of 32;
//   - flag derivation and the per-row plain mask, checked against a direct
//     definition, with the mask read exactly where the FP32 step kernel reads
//     it (its 4-word window from the word holding row y0 - 1 of every chunk,
//     guarded by the word count), through bounds-checked accesses;
//   - every argument check of lbm_init / lbm_batch_init / lbm_net_create that
//     runs before the first HIP call.
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <vector>

#include "lbm.h"
#include "lbm_internal.h"
#include "lbm_net.h"

namespace lbm {
void derive_flags_of(const lbm_params *p, const uint8_t *solid, std::vector<uint16_t> &out);
void row_plain_mask(int nx, int ny, const std::vector<uint16_t> &fl, std::vector<uint32_t> &mask);
}

static int failures = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::printf("CHECK failed at line %d: %s\n", __LINE__, #cond); \
            ++failures;                                                    \
        }                                                                  \
    } while (0)

static lbm_params base(int nx, int ny) {
    lbm_params p{};
    p.nx = nx; p.ny = ny; p.tau = 1.0; p.rho0 = 1.0;
    p.g_axis = -5.0 / 9; p.g_diag = -5.0 / 36; p.w_axis = -0.15; p.w_diag = -0.0375;
    p.rho_c = 1.0; p.f_elec = 1e-3; p.elec_layers = 2; p.elec_walls = 3u;
    p.storage = LBM_F32; p.collision = LBM_COLLIDE_BGK; p.trt_magic = 3.0 / 16;
    return p;
}

static std::vector<uint8_t> rough(int nx, int ny, unsigned seed) {
    std::vector<uint8_t> s((size_t)nx * ny, 0);
    for (int x = 0; x < nx; ++x) {
        seed = seed * 1103515245u + 12345u;
        const int h = (int)((seed >> 16) % 3u);
        for (int y = 0; y < ny; ++y)
            if (y == 0 || y == ny - 1 || ((x / 4) % 3 == 0 && (y <= h || y >= ny - 1 - h))) s[(size_t)y * nx + x] = 1;
    }
    return s;
}

// The rows the FP32 kernel reads from the plain mask for one chunk [y0, y1):
// words w0 .. w0 + 3 with w0 the word of row max(y0 - 1, 0), each only while
// it is below the word count.
static void kernel_window(const std::vector<uint32_t> &mask, int ny, int y0) {
    const unsigned nwords = ((unsigned)ny + 31u) >> 5;
    const unsigned w0 = (unsigned)(std::max(y0 - 1, 0) & ~31) >> 5;
    for (unsigned k = 0; k < 4; ++k)
        if (w0 + k < nwords) (void)mask.at(w0 + k);   // throws if out of range
}

static void check_lattice(int nx, int ny, int storage) {
    lbm_params p = base(nx, ny);
    p.storage = storage;
    const size_t ws = lbm_workspace_bytes(&p);
    CHECK(ws > 0);
    // room for two population buffers and the flags at least
    const size_t pitch = (size_t)(nx + 63) / 64 * 64;
    CHECK(ws >= 2 * 9 * pitch * ny * (storage == LBM_F32 ? 4 : 2) + pitch * ny * 2);
    const std::vector<uint8_t> solid = rough(nx, ny, (unsigned)(nx * 131 + ny));
    std::vector<uint16_t> fl;
    lbm::derive_flags_of(&p, solid.data(), fl);
    CHECK(fl.size() == (size_t)nx * ny);
    std::vector<uint32_t> mask;
    lbm::row_plain_mask(nx, ny, fl, mask);
    CHECK(mask.size() == (size_t)(ny + 31) / 32);
    for (int y = 0; y < ny; ++y) {
        const uint16_t plain = (uint16_t)(y >= ny / 2 ? lbm::FL_TOP : 0u);
        bool all = true;
        for (int x = 0; x < nx; ++x) all = all && fl[(size_t)y * nx + x] == plain;
        CHECK(((mask.at((size_t)y / 32) >> (y % 32)) & 1u) == (all ? 1u : 0u));
    }
    // every chunking the library can choose: 1 .. ny chunks of rows
    for (int chunks = 1; chunks <= ny; ++chunks)
        for (int c = 0; c < chunks; ++c) kernel_window(mask, ny, (int)(((int64_t)c * ny) / chunks));
}

int main() {
    const int sizes[][2] = {{3, 3}, {7, 5}, {64, 31}, {65, 32}, {100, 33}, {37, 63}, {130, 64}, {300, 65},
                            {64, 95}, {8, 97}, {256, 128}, {129, 200}};
    for (auto &s : sizes)
        for (int storage = 0; storage < 3; ++storage) {
            try {
                check_lattice(s[0], s[1], storage);
            } catch (const std::out_of_range &e) {
                std::printf("out of range for %dx%d: %s\n", s[0], s[1], e.what());
                ++failures;
            }
        }
    // argument checks before any HIP call
    lbm_params p = base(64, 32);
    std::vector<uint8_t> solid = rough(64, 32, 1);
    std::vector<double> rho(64 * 32, 1.5);
    lbm_sim *sim = nullptr;
    CHECK(lbm_init(nullptr, &p, solid.data(), rho.data(), nullptr, nullptr, nullptr, 0, nullptr) == LBM_EINVAL);
    CHECK(lbm_init(&sim, nullptr, solid.data(), rho.data(), nullptr, nullptr, nullptr, 0, nullptr) == LBM_EINVAL);
    CHECK(lbm_init(&sim, &p, nullptr, rho.data(), nullptr, nullptr, nullptr, 0, nullptr) == LBM_EINVAL);
    CHECK(lbm_init(&sim, &p, solid.data(), rho.data(), nullptr, nullptr, nullptr, 0, nullptr) == LBM_EINVAL);
    CHECK(lbm_init(&sim, &p, solid.data(), rho.data(), nullptr, nullptr, (void *)0x1000, 16, nullptr) == LBM_ENOMEM);
    CHECK(lbm_init(&sim, &p, solid.data(), rho.data(), nullptr, nullptr, (void *)0x1001, 1u << 30, nullptr) == LBM_EINVAL);
    rho[16 * 64 + 10] = -1.0;                      // a fluid node in the middle row
    CHECK(lbm_init(&sim, &p, solid.data(), rho.data(), nullptr, nullptr, (void *)0x1000, 1u << 30, nullptr) == LBM_EINVAL);
    CHECK(sim == nullptr);
    CHECK(lbm_last_error(nullptr) != nullptr);
    lbm_params bad = p;
    bad.tau = 0.5;
    CHECK(lbm_workspace_bytes(&bad) == 0);
    bad = p; bad.nx = 2;
    CHECK(lbm_workspace_bytes(&bad) == 0);
    bad = p; bad.rounding = LBM_ROUND_STOCHASTIC;
    CHECK(lbm_workspace_bytes(&bad) == 0);
    bad = p; bad.storage = 7;
    CHECK(lbm_workspace_bytes(&bad) == 0);
    for (int s = -6; s <= 1; ++s) CHECK(lbm_status_string(s) != nullptr);
    // batch layouts of uneven channels
    std::vector<lbm_params> ps;
    for (auto &s : sizes) ps.push_back(base(s[0], s[1]));
    CHECK(lbm_batch_workspace_bytes((int32_t)ps.size(), ps.data()) > 0);
    ps[3].tau = 0.4;
    CHECK(lbm_batch_workspace_bytes((int32_t)ps.size(), ps.data()) == 0);
    lbm_batch *b = nullptr;
    CHECK(lbm_batch_init(&b, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) == LBM_EINVAL);
    CHECK(lbm_batch_last_error(nullptr) != nullptr);
    // network sizing
    lbm_net_config cfg{};
    cfg.H = 64; cfg.W = 256; cfg.batch = 4; cfg.cin = 3; cfg.cout = 3;
    cfg.chans[0] = 32; cfg.chans[1] = 64; cfg.chans[2] = 128; cfg.chans[3] = 128; cfg.act_bf16 = 1;
    CHECK(lbm_net_param_count(&cfg) > 0);
    CHECK(lbm_net_workspace_bytes(&cfg) > 0);
    lbm_net_config badc = cfg;
    badc.H = 60;                                  // not a multiple of 8
    CHECK(lbm_net_workspace_bytes(&badc) == 0);
    lbm_net *net = nullptr;
    CHECK(lbm_net_create(&net, &badc, nullptr, 0, nullptr) == LBM_EINVAL);
    std::printf(failures ? "host sanitizer run: %d FAILED\n" : "host sanitizer run: ok\n", failures);
    return failures ? 1 : 0;
}
