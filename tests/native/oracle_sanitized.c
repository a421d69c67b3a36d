/*
 * Sanitizer driver for the FP64 oracle (test infrastructure).  Built by
 * tests/test_sanitizers.py with gcc -fsanitize=address,undefined and run on
 * the CPU: it includes the oracle's source, steps small lattices of ragged
 * sizes (rough walls, both collision operators, both electric-force
 * directions, layer depths 1-3) and calls every exported function, so that an
 * out-of-bounds access or undefined behaviour anywhere in them aborts the run.
 * It also checks that the mass stays constant, so a silently wrong step fails.
 */
#include "../../oracle/lbm_oracle.c"

#include <stdio.h>

static uint64_t sm_state;
static double uniform(void)            /* SplitMix64 (Steele, Lea, Flood 2014) */
{
    uint64_t z = (sm_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1.0p-53;
}

static int run_case(int nx, int ny, int collision, int normal, int layers, uint64_t seed)
{
    orc_params p;
    memset(&p, 0, sizeof p);
    p.nx = nx; p.ny = ny; p.tau = 0.9; p.rho0 = 1.0;
    p.g_axis = -5.0 / 9.0; p.g_diag = -5.0 / 36.0;
    p.w_axis = -0.1496; p.w_diag = -0.0374;
    p.rho_c = 1.0; p.f_elec = 2e-3; p.elec_layers = layers; p.elec_walls = 3u;
    p.accel_x = 1e-5; p.collision = collision; p.trt_magic = 3.0 / 16.0; p.elec_normal = normal;
    const size_t n = (size_t)nx * ny;
    uint8_t *solid = calloc(n, 1), *layer = calloc(n, 1), *top = calloc(n, 1), *code = calloc(n, 1);
    double *rho = malloc(n * sizeof(double)), *ux = calloc(n, sizeof(double)), *uy = calloc(n, sizeof(double));
    double *f = calloc(9 * n, sizeof(double)), *out = calloc((size_t)ny, sizeof(double));
    double *F = calloc(6 * n, sizeof(double));
    uint16_t *flags = calloc(n, sizeof(uint16_t));
    sm_state = seed;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            size_t i = (size_t)y * nx + x;
            /* flat walls, random steps of height up to 2 on both walls */
            int h = (int)(uniform() * 3.0);
            solid[i] = (y == 0 || y == ny - 1 || (x % 7 < 3 && (y <= h || y >= ny - 1 - h))) ? 1 : 0;
            rho[i] = solid[i] ? 0.0 : (y < 3 || y > ny - 4 ? 0.16 : 1.9) + 1e-3 * (uniform() - 0.5);
            if (!solid[i]) { ux[i] = 1e-3 * (uniform() - 0.5); uy[i] = 1e-3 * (uniform() - 0.5); }
        }
    orc_flags(&p, solid, flags);
    orc_electric_layer(&p, solid, layer, top);
    orc_electric_normal(&p, solid, code);
    orc_forces(&p, solid, rho, F, F + 2 * n, F + 4 * n);
    orc_init(&p, solid, rho, ux, uy, f);
    double Q0, M0, Q1, M1;
    orc_flux(&p, solid, f, &Q0, &M0);
    int bad = orc_step(&p, solid, f, 40);
    orc_flux(&p, solid, f, &Q1, &M1);
    orc_moments(&p, solid, f, rho, ux, uy);
    orc_profile(&p, solid, f, out);
    int fail = bad || !(fabs(M1 / M0 - 1.0) < 1e-12);
    printf("%dx%d collision %d normal %d layers %d: mass drift %.2e flux %.3e%s\n", nx, ny, collision, normal,
           layers, M1 / M0 - 1.0, Q1, fail ? "  FAIL" : "");
    free(solid); free(layer); free(top); free(code); free(rho); free(ux); free(uy);
    free(f); free(out); free(F); free(flags);
    return fail;
}

int main(void)
{
    int fail = 0;
    int32_t ex[9], ey[9], opp[9];
    double w[9], feq[9];
    orc_velocity_set(ex, ey, w, opp);
    orc_equilibrium(1.2, 0.01, -0.02, feq);
    (void)orc_phi(1.0, 0.5);
    (void)orc_trt_omega_minus(0.9, 3.0 / 16.0);
    const int sizes[][2] = {{3, 3}, {5, 4}, {17, 9}, {31, 33}, {37, 19}, {64, 31}};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s)
        for (int collision = 0; collision < 2; ++collision)
            for (int normal = 0; normal < 2; ++normal)
                fail |= run_case(sizes[s][0], sizes[s][1], collision, normal, 1 + (int)(s % 3), 17u + s);
    printf(fail ? "oracle sanitizer run: FAIL\n" : "oracle sanitizer run: ok\n");
    return fail;
}
