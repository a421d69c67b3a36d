// Internal interface between the host library (lbm_api.hip) and the kernels
// (lbm_kernels.hip).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Flag word of a node (the format lbm_geometry exports).
constexpr uint32_t FL_SOLID = 0x100u;  // S(x) = 1
constexpr uint32_t FL_LAYER = 0x200u;  // electric layer
constexpr uint32_t FL_TOP = 0x400u;    // top electrode side, n = (0, +1)
constexpr uint32_t FL_NSHIFT = 11u;     // bits 11-14: direction a of the electric force, 0 = electrode

// Geometry of the device arrays: planes [9][ny][pitch], flags [ny][pitch].
struct Grid {
    int32_t nx, ny;
    int32_t pitch;     // row pitch in elements (multiple of 64)
    uint32_t plane;    // elements per plane = ny * pitch
};

// Model constants in FP32 as the kernels use them.
struct Model {
    float tau, omega;          // omega = 1 / tau
    float rho0, log2e_inv_rho0;   // rho0 and log2(e) / rho0 (eq. (4) on the base-2 exponential)
    float rho_off;             // reference density of the stored deviations (0: raw f)
    float ga, gd, wa, wd;      // G_a and W_a per direction class
    float rho_c, f_elec;
    float f_elec_diag;         // f_elec / sqrt 2 (force along a diagonal face normal)
    float gx, gy;              // driving acceleration
    int32_t trt;               // 0: BGK with the velocity shift; 1: TRT, 2: MRT, with Guo forcing
    float omega_m;             // TRT: relaxation rate of the antisymmetric part (MRT: s_q)
    float mrt_se, mrt_seps;    // MRT: rates of the energy moments e and eps
    float src_p, src_m;        // TRT: source weights 1 - omega/2 and 1 - omega_m/2
    int32_t sround;            // 1: stochastic rounding of 16-bit stores (0: nearest)
};

struct StepArgs {
    const void *src;
    void *dst;
    const uint16_t *flags;
    Grid g;
    Model m;
    // Tiling: the lattice is cut into strips of block_x columns, each strip
    // into `chunks` chunks of consecutive rows (sizes differ by at most one);
    // tile t = strip * chunks + chunk.  Workgroup b runs tile
    // (b mod 8) * tiles_per_xcd + b / 8, so an XCD gets consecutive tiles.
    int32_t chunks;
    int32_t ntiles;
    int32_t tiles_per_xcd;
    // bit y of word y / 32: every node of row y has the plain flag word, 0 in
    // the bottom half (y < ny / 2) and FL_TOP in the top half
    const uint32_t *rowplain;
    // Stochastic rounding: two-slot step counter (slot par is this step's,
    // the kernel writes the next count to the other slot).
    uint32_t *rng;
    int32_t par;
    // Per-node acceleration field [2][ny][nx] (x plane, then y plane), added
    // to (gx, gy); NULL for none (fused kernel, BGK, nearest rounding only).
    const float *acc;
};

// One channel of a batch: its lattice, model and device arrays.
struct ChannelDesc {
    Grid g;
    Model m;
    int32_t chunks;            // row chunks per strip
    int32_t chunks_k;          // row chunks per strip of the multi-step batch kernel
    const void *buf[2];        // population buffers A and B
    const uint16_t *flags;
    const uint32_t *rowplain;  // bit y: every node of row y has the plain flag word (see lbm_kernels.hip)
};

// Persistent batched step: workgroups take tiles from a queue (one counter
// per step slot, zeroed before use) until the list is exhausted.  A tile is
// (channel << 16) | (strip * chunks + chunk).
struct BatchStepArgs {
    const ChannelDesc *descs;
    const uint32_t *tiles;
    uint32_t *counters;
    int32_t ntiles;
    int32_t slot;
    int32_t parity;            // index of the source buffer of every active channel
    int32_t trt;               // collision operator of every channel (Model::trt)
    int32_t sround;            // rounding of every channel (Model::sround)
    uint32_t *rng;             // two-slot step counter of stochastic rounding (slot parity is read)
};

// Launchers; each returns the hipError_t of its launch.
hipError_t launch_step(int storage, const StepArgs &a, int block_x, hipStream_t s);
// Resident workgroups of the step kernel per compute unit.
int step_blocks_per_cu(int storage, int block_x, bool trt, bool sr);
// The step kernel compiled for 8 waves per SIMD, and its resident workgroups.
hipError_t launch_step8(int storage, const StepArgs &a, int block_x, hipStream_t s);
int step8_blocks_per_cu(int storage, int block_x, bool trt, bool sr);
// k = 2 or 3 time steps per launch (src -> dst after k steps; strips of
// block_x - 2 (2k - 1) columns), its LDS per workgroup and its resident
// workgroups per compute unit.
hipError_t launch_stepk(int storage, const StepArgs &a, int block_x, int k, hipStream_t s);
size_t stepk_lds_bytes(int storage, int block_x, int k);
int stepk_blocks_per_cu(int storage, int block_x, int k, bool trt, bool sr);
// The split step (a producer wave streams rows into LDS for block_x compute
// threads; block_x = 128 or 256) and its resident workgroups per compute unit.
hipError_t launch_step_split(int storage, const StepArgs &a, int block_x, hipStream_t s);
int split_blocks_per_cu(int storage, int block_x);
// The wide step: v = 2 or 4 adjacent columns per thread, block_x threads per
// workgroup (block_x * v columns per strip).
hipError_t launch_step_wide(int storage, const StepArgs &a, int block_x, int v, hipStream_t s);
int wide_blocks_per_cu(int storage, int block_x, int v);
// f^eq(rho, u) on fluid nodes, stored as deviations from w_a * rho_off.
hipError_t launch_init(int storage, void *dst, const uint16_t *flags, const Grid &g, float rho_off,
                       const float *rho, const float *ux, const float *uy, int dense_pitch,
                       hipStream_t s);
hipError_t launch_fill(void *dst, size_t bytes, hipStream_t s);
// One-pass non-temporal copy of bytes (a multiple of 16): each lane moves
// per_lane (1, 2 or 4) chunks of 16 bytes.
hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, int per_lane, hipStream_t s);
hipError_t launch_round_sr(const float *in, const uint32_t *r, uint16_t *out, uint32_t n, int storage,
                           hipStream_t s);
hipError_t launch_moments(int storage, const void *src, const uint16_t *flags, const Grid &g,
                          float rho_off, float *rho, float *ux, float *uy, hipStream_t s);
// grid > 0: persistent kernel with that many workgroups taking tiles from the
// queue (counter a.slot); grid <= 0: one workgroup per tile (no counter).
hipError_t launch_batch_step(int storage, const BatchStepArgs &a, int block_x, int grid, hipStream_t s);
int batch_blocks_per_cu(int storage, int block_x, bool trt, bool sr);
// The batched step with k = 2 or 3 time steps per launch (k_batch_tilesk), one
// workgroup per tile of a.tiles (strips of block_x - 2(2k - 1) columns,
// ChannelDesc::chunks_k chunks per strip); block_x 256 or 512.
hipError_t launch_batch_stepk(int storage, const BatchStepArgs &a, int block_x, int k, hipStream_t s);
// Per-channel FP64 reduction of channels ids[0..n): out[4*k] = Q, out[4*k+1] =
// mass, out[4*k+2] = bad nodes, for the buffer index cur[ids[k]].
hipError_t launch_batch_reduce(int storage, const ChannelDesc *descs, const int32_t *ids,
                               const int32_t *cur, int n, double *out, hipStream_t s);
// FP64 reduction: out[0] = sum u_x, out[1] = sum rho, out[2] = number of bad
// nodes; partials must hold 4 * max_reduce_blocks() doubles.
int max_reduce_blocks();
// Workgroups (and FP64 partial quadruples) launch_reduce uses for a lattice.
int reduce_blocks(const Grid &g);
hipError_t launch_reduce(int storage, const void *src, const uint16_t *flags, const Grid &g,
                         float rho_off, double *partials, double *out, hipStream_t s);
// Channel-averaged u_x per row into out[ny] (device), one workgroup per row.
hipError_t launch_profile(int storage, const void *src, const uint16_t *flags, const Grid &g, float rho_off,
                          double *out, hipStream_t s);

}  // namespace lbm
