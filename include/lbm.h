/*
 * liblbm: D2Q9 Shan-Chen lattice Boltzmann with the electrowetting-on-dielectric
 * (EWOD) electric force, for AMD Instinct MI355X (gfx950).
 *
 * The model is the one of Li, Li, Chen & Fang, "Lattice Boltzmann simulation of
 * electrowetting-on-dielectric in a rough-wall channel" (arXiv:0708.4182):
 *   eq. (1)  BGK evolution f_a(x + e_a, t + 1) - f_a(x, t) = -(f_a - f_a^eq)/tau
 *   eq. (2)  rho = sum_a f_a,  rho u = sum_a f_a e_a
 *   eq. (3)  f_a^eq = w_a rho [1 + 3 e_a.u + 9/2 (e_a.u)^2 - 3/2 u^2]
 *   eq. (5)  F_sigma = -phi(x) sum_a G_a phi(x + e_a) e_a,  phi = rho0 (1 - exp(-rho/rho0))
 *   eq. (6)  F_w = -phi(x) sum_a W_a S(x + e_a) e_a
 *   eq. (9)  electric force f n on the conductive liquid (rho >= rho_c) in the
 *            layer next to the insulator, n pointing to the electrode
 *   eq. (10) rho u' = rho u + tau (F_sigma + F_w + f), u' enters f^eq in eq. (1)
 *   eq. (11) Q = (1/L) integral of u_x over the channel
 * Walls are solid nodes of a mask; populations arriving from a solid node are
 * replaced by halfway bounce-back.  The domain is periodic in x and y.
 * Two options are not the paper's and are off by default: a two-relaxation-
 * time collision with Guo's forcing term in place of eq. (10) and BGK
 * (lbm_params.collision), and the electric force along the local face normal
 * of a rough wall instead of towards the electrode (lbm_params.elec_normal).
 * 16-bit population storage and its stochastic rounding (lbm_params.storage,
 * lbm_params.rounding) are storage formats, not part of the model.
 *
 * Conventions for every entry point:
 *   - the return value is an lbm_status: 0 on success, < 0 on error; nothing
 *     throws across this interface;
 *   - host arrays are row-major [ny][nx] with x fastest; "device" pointers are
 *     HIP device addresses on the device current when lbm_init was called;
 *   - the caller owns every array it passes and the device workspace; the
 *     library copies what it needs during the call and never allocates device
 *     memory itself; it owns only the opaque handle;
 *   - all GPU work of a handle is issued on the HIP stream given to lbm_init;
 *     calls marked "asynchronous" return before the GPU finishes;
 *   - one handle must not be used from two threads at once;
 *   - after an error other than LBM_EINVAL the handle is in an error state
 *     (sticky) and every later call returns LBM_ESTATE until lbm_free.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,    /* bad argument or parameter; nothing was launched       */
    LBM_ENOMEM = -2,    /* workspace too small                                   */
    LBM_EDEVICE = -3,   /* a HIP call failed (message in lbm_last_error)         */
    LBM_EDIVERGED = -4, /* a fluid density became <= 0 or not finite             */
    LBM_ESTATE = -5     /* handle is in a sticky error state                     */
} lbm_status;

/* How populations are stored in device memory.  The arithmetic is FP32 in all
 * three cases.  Each format stores the deviation d_a = f_a - w_a rho_ref from the
 * rest populations of a reference density (lbm_params.rho_ref), rounded to
 * nearest even, and decodes f_a = w_a rho_ref + d_a in FP32. */
typedef enum { LBM_F32 = 0, LBM_F16 = 1, LBM_BF16 = 2 } lbm_storage;

/* Electrode walls (bit set): the electric layer exists only next to these. */
#define LBM_ELEC_BOTTOM 1u /* nodes with y <  ny/2, n = (0, -1) */
#define LBM_ELEC_TOP 2u    /* nodes with y >= ny/2, n = (0, +1) */

typedef struct {
    int32_t nx, ny;        /* lattice size; both >= 3                                  */
    double tau;            /* relaxation time of eq. (1); > 0.5                        */
    double rho0;           /* constant of the pseudopotential phi; > 0                 */
    double g_axis, g_diag; /* Green function G_a of eq. (5) for |e_a| = 1 and sqrt 2   */
    double w_axis, w_diag; /* fluid-wall strength W_a of eq. (6), same classes         */
    double rho_c;          /* critical density: fluid with rho >= rho_c is conductive  */
    double f_elec;         /* magnitude f of the electric force per layer node         */
    int32_t elec_layers;   /* layer = fluid within this Chebyshev distance of a solid  */
    uint32_t elec_walls;   /* LBM_ELEC_BOTTOM | LBM_ELEC_TOP                            */
    double accel_x, accel_y; /* driving acceleration g: body force rho g on every node */
    int32_t storage;       /* lbm_storage                                              */
    double rho_ref;        /* storage reference density (>= 0): populations are held as
                              d_a = f_a - w_a rho_ref; 0 selects the default, raw f for
                              LBM_F32 and rho0 for LBM_F16 / LBM_BF16.  A value near the
                              liquid density keeps the stored numbers small where the
                              flow is, which FP32 needs to resolve slow velocity modes  */
    int32_t collision;     /* LBM_COLLIDE_BGK: the paper's velocity shift, eq. (10), and
                              BGK relaxation, eq. (1).  LBM_COLLIDE_TRT_GUO and
                              LBM_COLLIDE_MRT_GUO (not in the paper): the same force F
                              with Guo's forcing term and a two- or multiple-
                              relaxation-time collision, see below                   */
    double trt_magic;      /* Lambda of LBM_COLLIDE_TRT_GUO and LBM_COLLIDE_MRT_GUO
                              (> 0; 3/16 puts halfway bounce-back walls exactly
                              halfway for plane Poiseuille flow at any tau); ignored
                              for LBM_COLLIDE_BGK                                     */
    int32_t elec_normal;   /* direction n of the electric force f n.  0: towards the
                              electrode wall, (0, -1) on the bottom half and (0, +1)
                              on the top half.  1: the local face normal of the
                              insulator: for a layer node at Chebyshev distance d from
                              the nearest solid node, the lattice direction
                              (sgn v_x, sgn v_y) of v = sum of (s - x) over the solid
                              nodes s at distance d, normalised (diagonals by
                              1/sqrt 2); the electrode direction where v = 0         */
    int32_t rounding;      /* rounding of the stored 16-bit deviations, see below:
                              LBM_ROUND_NEAREST (default) or LBM_ROUND_STOCHASTIC
                              (LBM_F16 and LBM_BF16 only; LBM_EINVAL with LBM_F32)    */
    double mrt_s_e, mrt_s_eps; /* LBM_COLLIDE_MRT_GUO: relaxation rates of the energy
                              moments e and eps, each in (0, 2) (Lallemand & Luo use
                              1.64 and 1.54); ignored by the other operators         */
} lbm_params;

/* Rounding of 16-bit storage (lbm_params.rounding).  LBM_ROUND_NEAREST rounds
 * every stored deviation to nearest even.  Where the flow is nearly steady a
 * node's post-collision values repeat from step to step, so do their rounding
 * errors, and the mass they add or remove grows linearly with time (a droplet
 * at rest can gain 10% in 20,000 steps).  LBM_ROUND_STOCHASTIC rounds each
 * value up or down with probabilities that make the expected stored value
 * exact: the magnitude rounds up when 16 random bits added below the result's
 * last place carry into it (for FP16 the top 13 of them on normal values).
 * The bits are a counter-based hash (lowbias32) of the node's offset in its
 * population plane and the number of steps taken, so runs are reproducible:
 * the same calls give bitwise the same results, hipGraph replays equal eager
 * steps, and a channel of a batch equals the same lattice run alone.  Mass
 * errors then grow like the square root of the step count.  Runs in
 * LBM_KERNEL_FUSED and LBM_KERNEL_FUSED8 only; lbm_load_state restarts the
 * count at the state's step number.
 * Fitness for runs of ~20,000 steps towards a steady state (128 x 64 droplet,
 * 512 x 128 rough channel, against the FP64 model): LBM_F32 holds the angle
 * to 0.001 degree and the mass to 1e-5; LBM_F16 + stochastic to 0.05 degree,
 * 1e-3 of the mass and 1.4e-4 of the flux; LBM_BF16 + stochastic to 0.5
 * degree, 1.5e-3 of the mass and 5e-3 of the flux.  With nearest rounding the
 * 16-bit formats drift (FP16: +11% mass, 1.7 degrees; BF16: the droplet falls
 * apart, the flux is 38% off): fit for short transients and throughput
 * measurements only. */
#define LBM_ROUND_NEAREST 0
#define LBM_ROUND_STOCHASTIC 1

/* Collision operators (lbm_params.collision).  LBM_COLLIDE_TRT_GUO: the
 * equilibrium of eq. (3) takes u = (sum f e + F/2) / rho; the symmetric and
 * antisymmetric parts of f - f^eq relax at omega+ = 1/tau and omega- with
 * (1/omega+ - 1/2)(1/omega- - 1/2) = trt_magic; the source
 * S_a = w_a [3 (e_a - u) + 9 (e_a . u) e_a] . F of Guo, Zheng & Shi (2002)
 * is split the same way and weighted (1 - omega+/2), (1 - omega-/2).  F is the
 * total force of eq. (10) (eqs. (5), (6), the electric force and rho g).
 * lbm_moments and lbm_flux report u = sum f e / rho of eq. (2) for both. */
#define LBM_COLLIDE_BGK 0
#define LBM_COLLIDE_TRT_GUO 1
/* LBM_COLLIDE_MRT_GUO: multiple-relaxation-time collision in the orthogonal
 * moment basis m = M f = (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy) of
 * Lallemand & Luo (Phys. Rev. E 61, 6546, 2000), with the same u, F and Guo
 * source as TRT taken to moment space: m* = m - S (m - M f^eq) + (I - S/2) M S,
 * S = diag(0, mrt_s_e, mrt_s_eps, 0, s_q, 0, s_q, 1/tau, 1/tau), s_q = omega-
 * of the TRT relation; f* = M^-1 m*.  Shear viscosity (tau - 1/2)/3, bulk
 * viscosity (1/mrt_s_e - 1/2)/3; with mrt_s_e = mrt_s_eps = 1/tau it is
 * LBM_COLLIDE_TRT_GUO.  Runs wherever TRT runs (the same kernels). */
#define LBM_COLLIDE_MRT_GUO 2

typedef struct lbm_sim lbm_sim;

/* Bytes of device workspace lbm_init needs for these parameters (0 if the
 * parameters are invalid).  The workspace holds two population buffers, the
 * per-node flag words and reduction scratch. */
size_t lbm_workspace_bytes(const lbm_params *p);

/*
 * Create a simulation.  solid: host uint8 [ny][nx], 1 = solid node (the paper's
 * S = 1).  rho_init, ux_init, uy_init: host float64 [ny][nx]; the velocities may
 * be NULL (rest).  Populations start at f_a^eq(rho_init, u_init) of eq. (3) on
 * fluid nodes.  dev_ws: device workspace of ws_bytes >= lbm_workspace_bytes(p),
 * 256-byte aligned, owned by the caller, not touched by anything else while
 * the handle lives.  stream: hipStream_t (NULL = default stream).
 * Validates everything before any GPU work: nx, ny >= 3; tau > 0.5; rho0 > 0;
 * at least one fluid node; storage valid; elec_layers >= 0; finite values.
 * Synchronizes the stream before returning.  On success *out is a new handle.
 */
lbm_status lbm_init(lbm_sim **out, const lbm_params *p, const uint8_t *solid,
                    const double *rho_init, const double *ux_init, const double *uy_init,
                    void *dev_ws, size_t ws_bytes, void *stream);

/* Re-initialise the populations of an existing handle to f^eq(rho, u) from
 * device float32 fields [ny][nx] (e.g. a predicted steady state used as a
 * warm start).  Geometry and parameters are kept.  Asynchronous. */
lbm_status lbm_init_device(lbm_sim *sim, const float *rho, const float *ux, const float *uy);

/* Advance nsteps >= 0 full time steps of eq. (1) (collision with the forces of
 * eqs. (5), (6), (9), (10), then streaming with bounce-back).  Asynchronous. */
lbm_status lbm_step(lbm_sim *sim, int64_t nsteps);

/* Density and velocity of eq. (2) (u before the force shift of eq. (10)) of
 * the current state, as float32 [ny][nx]; solid nodes give 0.  on_device != 0:
 * the three pointers are device arrays and the call is asynchronous; else they
 * are host arrays and the call synchronizes.  Any pointer may be NULL. */
lbm_status lbm_moments(lbm_sim *sim, float *rho, float *ux, float *uy, int on_device);

/* Flux of eq. (11) with L = nx, Q = (1/nx) sum over fluid nodes of u_x, and the
 * total fluid mass M = sum of rho, both accumulated in FP64 on the GPU in a
 * fixed order (bitwise reproducible).  Synchronizes.  Returns LBM_EDIVERGED
 * (sticky) if any fluid density is <= 0 or not finite; Q and M are still set. */
lbm_status lbm_flux(lbm_sim *sim, double *Q, double *M);

/* lbm_flux for callers that cannot allocate device memory (code under hipGraph
 * capture nearby, serving loops, harnesses that forbid allocation): the same
 * kernels, bitwise the same Q and M, but the FP64 reduction's partial sums and
 * result live in a library-owned static device array (32 KiB + 256 B per
 * device, held until the process ends) instead of the handle's workspace.
 * Allocates nothing.  Every call on one device shares that device's array:
 * calls that overlap on one device (two streams, two threads) race and must
 * be serialised by the caller.  LBM_EDEVICE if the array's address could not
 * be found at lbm_init; LBM_EINVAL if the reduction would need more partial
 * sums than the array holds (it never does: at most 1024 workgroups).
 * Synchronizes; LBM_EDIVERGED as lbm_flux. */
lbm_status lbm_flux_static(lbm_sim *sim, double *Q, double *M);

/* Channel-averaged velocity profile: ux_mean[y] = (1/nx) sum over the fluid
 * nodes of row y of u_x from eq. (2) (the profile of the paper's velocity
 * figure), host float64 [ny], accumulated in FP64 on the GPU in a fixed order;
 * its sum over the rows is the flux Q of lbm_flux up to summation order.
 * Synchronizes. */
lbm_status lbm_profile(lbm_sim *sim, double *ux_mean);

/* Per-node flag words (host uint16 [ny][nx]): bit (a-1) = S(x + e_a) for
 * a = 1..8 with e_1..e_8 = (1,0),(0,1),(-1,0),(0,-1),(1,1),(-1,1),(-1,-1),(1,-1);
 * bit 8 = S(x); bit 9 = electric layer; bit 10 = top electrode side; bits
 * 11-14 = a in 1..8 where the electric force acts along e_a (elec_normal = 1),
 * else 0.  A solid node is exactly 0x100.  Synchronizes. */
lbm_status lbm_geometry(lbm_sim *sim, uint16_t *flags);

/* Change the electric force magnitude and the driving acceleration without
 * re-initialising (parameter sweeps).  Takes effect at the next lbm_step. */
lbm_status lbm_set_forces(lbm_sim *sim, double f_elec, double accel_x, double accel_y);

/* Per-node acceleration field: acc is a device float32 array [2][ny][nx]
 * (the x components, then the y components; NULL removes the field).  Each
 * fluid node then feels the body force rho (g + acc(x)) in place of rho g,
 * through the velocity shift of eq. (10).  It carries forces that act on the
 * fluid's mass in a prescribed pattern, such as the artificial attraction the
 * paper applies to gather a homogeneous fluid into one droplet in the middle
 * of the substrate before releasing it (the droplet run of its EWOD section).
 * The caller owns acc and keeps it unchanged and alive while it is set (the
 * kernels read it at every step).  Runs in LBM_KERNEL_FUSED with
 * LBM_COLLIDE_BGK and nearest rounding only (LBM_EINVAL otherwise, also
 * from lbm_set_kernel and lbm_autotune while a field is set).  Takes effect
 * at the next lbm_step; drops captured graphs. */
lbm_status lbm_set_accel_field(lbm_sim *sim, const float *acc);

/* Kernel tile: block_x columns per workgroup (64, 128, 256 or 512; 128 or 256
 * for the split kernel) and about
 * rows_per_block rows marched by one workgroup; 0 picks as many row chunks as
 * fill one wave of resident workgroups (chunks of at least 8 rows).  Results
 * do not depend on the tile (bitwise).  Default 256 x 0.  Takes effect at the
 * next lbm_step. */
lbm_status lbm_set_tile(lbm_sim *sim, int32_t block_x, int32_t rows_per_block);

/* Step kernel.  LBM_KERNEL_FUSED: every thread loads, computes and stores its
 * column.  LBM_KERNEL_WIDE2 / LBM_KERNEL_WIDE4: the same with 2 or 4 adjacent
 * columns per thread, so each plane moves as 2 or 4 values per lane (a strip
 * of block_x threads covers 2 or 4 x block_x columns).  LBM_KERNEL_SPLIT: one
 * producer wave per workgroup streams the pulled rows into LDS two rows ahead
 * with direct-to-LDS loads and block_x compute threads only read LDS and store
 * (block_x 128 or 256; selecting it with another block_x sets block_x to 128).
 * LBM_KERNEL_FUSED8: the fused kernel compiled for 8 resident waves per SIMD
 * (64 registers; a few loop invariants live in scratch memory) instead of 7.
 * LBM_KERNEL_TWO / LBM_KERNEL_THREE: two or three time steps per launch
 * (temporal blocking): each step's results stay in LDS, in the storage
 * format, for the next, so the populations cross HBM once per two or three
 * steps; a workgroup of block_x threads (256 or 512; selecting one with a
 * smaller block_x sets 256, and a block_x whose LDS exceeds the device's
 * per-workgroup limit is refused) yields block_x - 6 or block_x - 10
 * columns, and the nsteps mod 2 (or 3) remaining steps of an lbm_step call
 * run the fused kernel.  Every lbm_step call still ends on the exact state
 * after nsteps.
 * All give bitwise the same results.  Default LBM_KERNEL_FUSED.  Takes effect
 * at the next lbm_step.  With LBM_COLLIDE_TRT_GUO, LBM_COLLIDE_MRT_GUO or
 * LBM_ROUND_STOCHASTIC only LBM_KERNEL_FUSED, LBM_KERNEL_FUSED8, LBM_KERNEL_TWO and
 * LBM_KERNEL_THREE are accepted (LBM_EINVAL otherwise) and tuned. */
#define LBM_KERNEL_FUSED 0
#define LBM_KERNEL_SPLIT 1
#define LBM_KERNEL_WIDE2 2
#define LBM_KERNEL_WIDE4 3
#define LBM_KERNEL_FUSED8 4
#define LBM_KERNEL_TWO 5
#define LBM_KERNEL_THREE 6
lbm_status lbm_set_kernel(lbm_sim *sim, int32_t kernel);

/* Replay steps as hipGraphs: lbm_step(n) runs floor(n / steps_per_graph)
 * replays of a captured graph of steps_per_graph launches, then the remainder
 * as ordinary launches.  steps_per_graph: 0 (ordinary launches only, the
 * default) or an even number in [2, 4096].  A graph is captured on a private
 * stream at the first replay from each buffer parity and holds kernel launches
 * only; it bakes in the tile, kernel and forces, so lbm_set_tile,
 * lbm_set_kernel, lbm_set_forces and lbm_autotune drop it.  Results are
 * bitwise those of ordinary launches.  Worth it for small lattices, whose
 * steps are bound by launch overhead. */
lbm_status lbm_set_graph(lbm_sim *sim, int32_t steps_per_graph);

/* The current kernel, block_x and rows_per_block (any pointer may be NULL). */
lbm_status lbm_get_tile(const lbm_sim *sim, int32_t *kernel, int32_t *block_x, int32_t *rows_per_block);

/* Autotuner: times each candidate (fused kernels: block_x in 64..512 (6 waves)
 * or 128..512 (8 waves); wide
 * kernels: block_x 64..256; split kernel: block_x 128 or 256; rows_per_block
 * in {0, 4, 8, 16, 32, 64, 128}) for `reps`
 * launches on the current state and keeps the fastest.  The trial launches
 * write only the spare population buffer, so the simulation state and step
 * count are unchanged.  Synchronizes.  The chosen tile and its time per step
 * (microseconds) are returned through the non-NULL pointers; lbm_get_tile
 * tells the chosen kernel. */
lbm_status lbm_autotune(lbm_sim *sim, int32_t reps, int32_t *block_x, int32_t *rows_per_block,
                        float *us_per_step);

/* Checkpoint: raw device state (stored populations + step counter) to/from a
 * host buffer of lbm_state_bytes(sim) bytes.  Both synchronize.  Loading a
 * saved state and stepping gives bitwise the same result as never stopping. */
size_t lbm_state_bytes(const lbm_sim *sim);
lbm_status lbm_save_state(lbm_sim *sim, void *host, size_t bytes);
lbm_status lbm_load_state(lbm_sim *sim, const void *host, size_t bytes);

/* ------------------------------------------------------------------------
 * Batched engine: n independent lattices ("channels") of uneven sizes, each
 * with its own parameters and geometry (the paper's sweeps over field
 * strength, channel width and roughness, Figs. 3, 5-8).  Every time step is
 * one kernel launch over the tiles of all active channels: by default one
 * workgroup per tile, or a persistent grid whose workgroups take tiles from a
 * queue (lbm_batch_set_schedule); K steps can be captured as one hipGraph and
 * replayed.  With lbm_batch_set_kernel a launch can advance the batch by two
 * or three steps (k_stepk's temporal blocking on each channel's tiles).
 * Conventions as above; all channels share one storage format, collision
 * operator and rounding (LBM_EINVAL otherwise); all active channels advance
 * together.  A retired channel keeps its last state and is
 * no longer stepped.
 * ------------------------------------------------------------------------ */
typedef struct lbm_batch lbm_batch;

/* Device workspace for the batch (0 if any parameter set is invalid). */
size_t lbm_batch_workspace_bytes(int32_t n, const lbm_params *p /* [n] */);

/* Create a batch.  p, solid, rho_init: arrays of n entries (host), channel i
 * with arrays [ny_i][nx_i] as for lbm_init; ux_init / uy_init may be NULL or
 * contain NULL entries.  Validation as for lbm_init, per channel, before any
 * GPU work.  Synchronizes. */
lbm_status lbm_batch_init(lbm_batch **out, int32_t n, const lbm_params *p, const uint8_t *const *solid,
                          const double *const *rho_init, const double *const *ux_init,
                          const double *const *uy_init, void *dev_ws, size_t ws_bytes, void *stream);

/* Advance every active channel by nsteps time steps.  With a graph length K
 * (lbm_batch_set_graph) the steps run as hipGraph replays of K steps, the
 * remainder eagerly.  Under a multi-step kernel (lbm_batch_set_kernel) a run
 * of steps is floor(steps / k) k-step launches followed by single-step
 * launches for the rest.  Asynchronous. */
lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Flux Q_i (eq. (11), L = nx_i) and mass M_i of every channel, FP64, fixed
 * reduction order.  Synchronizes.  Returns LBM_EDIVERGED (not sticky) if any
 * channel has a density <= 0 or not finite; its Q_i is NaN. */
lbm_status lbm_batch_flux(lbm_batch *b, double *Q /* [n] */, double *M /* [n] */);

/* eq. (2) moments of channel i, as lbm_moments. */
lbm_status lbm_batch_moments(lbm_batch *b, int32_t i, float *rho, float *ux, float *uy, int on_device);

/* Velocity profile of channel i, as lbm_profile (host float64 [ny_i]). */
lbm_status lbm_batch_profile(lbm_batch *b, int32_t i, double *ux_mean);

/* Flag words of channel i, as lbm_geometry. */
lbm_status lbm_batch_geometry(lbm_batch *b, int32_t i, uint16_t *flags);

/* Re-initialise channel i to f^eq(rho, u) from device float32 fields
 * [ny_i][nx_i] (warm start); its step count restarts at 0.  Asynchronous. */
lbm_status lbm_batch_init_device(lbm_batch *b, int32_t i, const float *rho, const float *ux, const float *uy);

/* Change the electric force and driving acceleration of channel i. */
lbm_status lbm_batch_set_forces(lbm_batch *b, int32_t i, double f_elec, double accel_x, double accel_y);

/* Stop stepping the channels with done[i] != 0 (host uint8 [n]); rebuilds the
 * tile list.  Synchronizes. */
lbm_status lbm_batch_retire(lbm_batch *b, const uint8_t *done);

/* Tile shape: block_x columns (64..512) by about rows_per_tile rows (>= 8).
 * Results do not depend on it (bitwise).  Default 256 x 32. */
lbm_status lbm_batch_set_tile(lbm_batch *b, int32_t block_x, int32_t rows_per_tile);

/* Work distribution of a step launch: persistent != 0 runs a persistent grid
 * (resident workgroups take tiles from an atomic queue until it is empty);
 * 0 launches one workgroup per tile and lets the hardware dispatcher balance.
 * Results are bitwise the same.  Default 0. */
lbm_status lbm_batch_set_schedule(lbm_batch *b, int32_t persistent);

/* Steps per launch: LBM_KERNEL_FUSED (one; default), LBM_KERNEL_TWO or
 * LBM_KERNEL_THREE (two or three steps per launch from one workgroup per
 * tile, strips of block_x - 6 or block_x - 10 output columns, block_x 512 if
 * lbm_batch_set_tile chose 512, else 256).  Bitwise the same results as the
 * one-step kernel, for every storage format, operator and rounding mode.
 * LBM_EINVAL for another value.  Rebuilds the tile list; synchronizes. */
lbm_status lbm_batch_set_kernel(lbm_batch *b, int32_t kernel);

/* Current steps-per-launch setting as an LBM_KERNEL_* value (-1 for NULL). */
int32_t lbm_batch_get_kernel(const lbm_batch *b);

/* Time steps per captured graph: 0 (eager launches) or an even number up to
 * 1024.  Default 0. */
lbm_status lbm_batch_set_graph(lbm_batch *b, int32_t steps_per_graph);

/* Autotuner for the batch: schedule (persistent or one workgroup per tile) x
 * block_x x rows in {16, 32, 64} for the one-step kernel, and the two- and
 * three-step kernels at block_x 256 and 512 x the same rows; keeps the
 * fastest time per step (its kernel, schedule and tile shape stay set;
 * lbm_batch_get_kernel reports the kernel).  Trial launches write only the
 * spare buffers, so the state is unchanged. */
lbm_status lbm_batch_autotune(lbm_batch *b, int32_t reps, int32_t *block_x, int32_t *rows_per_tile,
                              float *us_per_step);

/* Steps taken by channel i (-1 for a bad index). */
int64_t lbm_batch_steps_done(const lbm_batch *b, int32_t i);

/* Free the handle (not the workspace). */
void lbm_batch_free(lbm_batch *b);

/* Last error message of the batch (or of the last failed lbm_batch_init if b
 * is NULL). */
const char *lbm_batch_last_error(const lbm_batch *b);

/* Measurement reference, not part of the model: copy `bytes` (a multiple of
 * 16; device pointers 16-byte aligned, not overlapping) from src to dst in one
 * pass of short-lived workgroups of 256 threads, each lane moving per_lane
 * (1, 2 or 4) chunks of 16 bytes with non-temporal loads and stores.  Its
 * rate is the practical HBM ceiling the step kernels are compared with.
 * Asynchronous on `stream`; LBM_EINVAL for bad arguments (message in
 * lbm_last_error(NULL)). */
lbm_status lbm_stream_copy(void *dst, const void *src, size_t bytes, int32_t per_lane, void *stream);

/* The stochastic rounding the step kernels apply to 16-bit stores
 * (LBM_ROUND_STOCHASTIC), value by value, for checking the encoder itself:
 * out[i] = in[i] rounded to FP16 (storage LBM_F16) or BF16 (LBM_BF16) with the
 * random bits r[i] (its low 13 bits for FP16, 16 for BF16): the bits are added
 * below the result's last place (for FP16 subnormal results, at the top of the
 * longer dropped field; below 2^-24 the result is 0 or 2^-24) and the word is
 * truncated, so the magnitude rounds up with probability (dropped part) /
 * (last place); Inf and NaN are converted as they are.  out holds the 16-bit
 * patterns.  Device pointers, n in [0, 2^32); asynchronous on `stream`;
 * LBM_EINVAL for another storage or a NULL pointer with n > 0 (message in
 * lbm_last_error(NULL)). */
lbm_status lbm_round_sr(const float *in, const uint32_t *r, uint16_t *out, int64_t n, int32_t storage, void *stream);

/* Time steps taken since lbm_init (or the loaded checkpoint). */
int64_t lbm_steps_done(const lbm_sim *sim);

/* Free the handle (not the workspace, which the caller owns).  NULL is a no-op. */
void lbm_free(lbm_sim *sim);

/* Last error message of a handle (or of the last failed lbm_init if sim is
 * NULL); never NULL. */
const char *lbm_last_error(const lbm_sim *sim);

/* Name of a status code. */
const char *lbm_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* LBM_H */
