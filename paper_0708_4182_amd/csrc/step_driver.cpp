// Standalone driver of liblbm for profiler runs (rocprofv3 kernel traces and
// counter passes): no Python, no torch.  It reads a lattice written by
// paper_0708_4182_amd/profile_case.py (parameters, solid mask, initial
// density), allocates the workspace, and for each storage format given runs
// `warmup` + `steps` steps at a fixed kernel and tile, then copies one FP32
// population buffer with lbm_stream_copy (the known-size calibration
// dispatch of counter passes).  Prints the mean time per step from HIP
// events.
//
//   step_driver CASE_FILE STEPS WARMUP KERNEL BLOCK_X ROWS STORAGE [STORAGE...]
//   (KERNEL: 0 fused, 4 fused8; STORAGE: 0 FP32, 1 FP16, 2 BF16)
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "lbm.h"

#define HCHECK(x)                                                                  \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            std::fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));          \
            return 1;                                                              \
        }                                                                          \
    } while (0)
#define LCHECK(x)                                                                  \
    do {                                                                           \
        lbm_status s_ = (x);                                                       \
        if (s_ != LBM_OK) {                                                        \
            std::fprintf(stderr, "%s: %s\n", #x, lbm_status_string(s_));          \
            return 1;                                                              \
        }                                                                          \
    } while (0)

int main(int argc, char **argv) {
    if (argc < 8) {
        std::fprintf(stderr, "usage: %s CASE STEPS WARMUP KERNEL BLOCK_X ROWS STORAGE [STORAGE...]\n", argv[0]);
        return 2;
    }
    FILE *fh = std::fopen(argv[1], "rb");
    if (!fh) {
        std::fprintf(stderr, "cannot open %s\n", argv[1]);
        return 2;
    }
    lbm_params p{};
    int32_t dims[2];
    if (std::fread(dims, sizeof dims, 1, fh) != 1 || std::fread(&p, sizeof p, 1, fh) != 1) return 2;
    const size_t n = (size_t)dims[0] * dims[1];
    if (dims[0] != p.nx || dims[1] != p.ny || n == 0) return 2;
    std::vector<uint8_t> solid(n);
    std::vector<double> rho(n);
    if (std::fread(solid.data(), 1, n, fh) != n || std::fread(rho.data(), sizeof(double), n, fh) != n) return 2;
    std::fclose(fh);
    const long steps = std::atol(argv[2]), warmup = std::atol(argv[3]);
    const int kernel = std::atoi(argv[4]), bx = std::atoi(argv[5]), rows = std::atoi(argv[6]);
    hipStream_t st;
    HCHECK(hipStreamCreate(&st));
    hipEvent_t e0, e1;
    HCHECK(hipEventCreate(&e0));
    HCHECK(hipEventCreate(&e1));
    for (int a = 7; a < argc; ++a) {
        p.storage = std::atoi(argv[a]);
        const size_t ws = lbm_workspace_bytes(&p);
        if (!ws) return 2;
        void *dws = nullptr;
        HCHECK(hipMalloc(&dws, ws));
        lbm_sim *sim = nullptr;
        LCHECK(lbm_init(&sim, &p, solid.data(), rho.data(), nullptr, nullptr, dws, ws, st));
        LCHECK(lbm_set_kernel(sim, kernel));
        LCHECK(lbm_set_tile(sim, bx, rows));
        LCHECK(lbm_step(sim, warmup));
        HCHECK(hipStreamSynchronize(st));
        HCHECK(hipEventRecord(e0, st));
        LCHECK(lbm_step(sim, steps));
        HCHECK(hipEventRecord(e1, st));
        HCHECK(hipEventSynchronize(e1));
        float ms = 0.f;
        HCHECK(hipEventElapsedTime(&ms, e0, e1));
        double Q = 0, M = 0;
        LCHECK(lbm_flux(sim, &Q, &M));
        std::printf("storage %d kernel %d tile %dx%d: %.4f ms per step over %ld steps; Q %.9e M %.9e\n", p.storage,
                    kernel, bx, rows, ms / (double)steps, steps, Q, M);
        lbm_free(sim);
        HCHECK(hipFree(dws));
    }
    // calibration dispatch: one FP32 population buffer, 9 nx ny 4 bytes each way
    const size_t cb = (size_t)9 * n * 4;
    void *a = nullptr, *b = nullptr;
    HCHECK(hipMalloc(&a, cb));
    HCHECK(hipMalloc(&b, cb));
    HCHECK(hipMemsetAsync(a, 0, cb, st));
    for (int k = 0; k < 3; ++k) LCHECK(lbm_stream_copy(b, a, cb, 1, st));
    HCHECK(hipStreamSynchronize(st));
    std::printf("calibration copy: %zu bytes x 3\n", cb);
    HCHECK(hipFree(a));
    HCHECK(hipFree(b));
    HCHECK(hipStreamDestroy(st));
    std::fflush(stdout);
    return 0;
}
