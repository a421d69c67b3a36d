/*
 * Oracle: plain, slow FP64 CPU implementation of the EWOD lattice Boltzmann
 * step.  TEST INFRASTRUCTURE ONLY: it exists to check the GPU library, it is
 * not part of the product path, and it shares no code with it.
 *
 * Model (Li, Li, Chen & Fang, "Lattice Boltzmann simulation of
 * electrowetting-on-dielectric in a rough-wall channel", arXiv:0708.4182):
 *   - D2Q9 velocities e_alpha and BGK evolution, eq. (1);
 *   - density and velocity as moments of f, eq. (2);
 *   - equilibrium with weights 4/9, 1/9, 1/36, eq. (3);
 *   - Shan-Chen interparticle force with pseudopotential
 *     phi = rho0 (1 - exp(-rho/rho0)) and Green function G_alpha, eq. (5);
 *   - fluid-wall force with W_alpha and the solid indicator S, eq. (6);
 *   - electric force f n on the conductive (rho >= rho_c) liquid in the layer
 *     next to the insulator, n pointing to the electrode, eq. (9) and the text
 *     around the critical density;
 *   - velocity shift rho u' = rho u + tau (F_sigma + F_w + f), eq. (10);
 *   - flux Q = (1/L) sum of u_x over the channel, eq. (11).
 *
 * Readings where the paper is silent (each one is a parameter or a stated rule):
 *   - the Green function is given per direction class (g_axis for |e| = 1,
 *     g_diag for |e| = sqrt 2), likewise the wall strength (w_axis, w_diag);
 *   - F_sigma sums over fluid neighbours only; solid neighbours enter through F_w;
 *   - walls use halfway bounce-back: a population that would stream from a
 *     solid node is replaced by the opposite post-collision population of the
 *     node itself;
 *   - the electric layer is every fluid node within Chebyshev distance
 *     elec_layers of a solid node, on the half of the domain (y < ny/2: bottom,
 *     else top) whose wall is an electrode; n = -y at the bottom, +y at the top;
 *   - a driving acceleration g adds F_b = rho g to the force of eq. (10);
 *   - the domain is periodic in x and y; walls are solid rows in the mask.
 *
 * Optionally (elec_normal = 1) the electric force acts along the local face
 * normal of the insulator instead of towards the flat electrode: for a layer
 * node x at Chebyshev distance d from the nearest solid node, v = sum of
 * (s - x) over the solid nodes s at exactly that distance, and n is the unit
 * lattice direction (sgn v_x, sgn v_y); if v = 0, n falls back to the
 * electrode direction.  On flat walls this is the electrode direction.
 *
 * A second collision operator, not in the paper, can replace steps 3-4 of the
 * step (collision = 1): two-relaxation-time (TRT) collision (Ginzburg 2005;
 * Ginzburg, Verhaeghe & d'Humieres 2008) with the forcing term of Guo, Zheng &
 * Shi (Phys. Rev. E 65, 046308, 2002).  The force is the same F of eq. (10);
 * the equilibrium takes u = (sum f e + F/2) / rho, the symmetric and
 * antisymmetric parts of f - f^eq relax at omega+ = 1/tau and omega- with
 * (1/omega+ - 1/2)(1/omega- - 1/2) = Lambda (trt_magic), and the source
 * S_a = w_a [3 (e_a - u) + 9 (e_a . u) e_a] . F enters split the same way,
 * weighted (1 - omega+/2) and (1 - omega-/2).
 *
 * A third (collision = 2), also not in the paper: multiple-relaxation-time
 * (MRT) collision in the orthogonal moment basis of Lallemand & Luo (Phys.
 * Rev. E 61, 6546, 2000), m = (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy),
 * with the same Guo forcing in moment space (Guo & Zheng 2008):
 * m* = m - S (m - m^eq) + (I - S/2) M S, where m^eq = M f^eq(rho, u) with
 * u = (sum f e + F/2) / rho, S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, 1/tau,
 * 1/tau), s_q = omega- of the TRT relation above (so Lambda keeps its
 * meaning), and f* = M^-1 m*.  With s_e = s_eps = 1/tau it is the TRT
 * operator; s_e sets the bulk viscosity, s_eps a kinetic mode.
 *
 * Arrays are row-major [ny][nx]; populations are planes [9][ny][nx].
 * Solid nodes carry no populations (their entries are ignored and left 0).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t nx, ny;
    double tau, rho0;
    double g_axis, g_diag;
    double w_axis, w_diag;
    double rho_c;
    double f_elec;
    int32_t elec_layers;
    uint32_t elec_walls; /* bit 0: bottom wall is an electrode, bit 1: top */
    double accel_x, accel_y;
    int32_t collision;   /* 0: BGK with the velocity shift of eq. (10); 1: TRT with Guo forcing */
    double trt_magic;    /* Lambda of the TRT operator (and of MRT's s_q) */
    int32_t elec_normal; /* 0: n towards the electrode wall; 1: local face normal */
    double mrt_s_e, mrt_s_eps; /* MRT rates of the energy moments e and eps */
} orc_params;

/* ---------------------------------------------------------------- lattice */
static int E[9][2];     /* e_alpha, built from the paper's trigonometric definition */
static double WT[9];    /* w_alpha of eq. (3) */
static int OPP[9];      /* e_opp(alpha) = -e_alpha */
static int lattice_ready = 0;

static void lattice_init(void)
{
    if (lattice_ready) return;
    const double pi = 3.14159265358979323846;
    E[0][0] = 0; E[0][1] = 0;
    for (int a = 1; a <= 4; ++a) {
        E[a][0] = (int)lround(cos(pi * (a - 1) / 2.0));
        E[a][1] = (int)lround(sin(pi * (a - 1) / 2.0));
    }
    for (int a = 5; a <= 8; ++a) {
        E[a][0] = (int)lround(sqrt(2.0) * cos(pi * (2 * a - 1) / 4.0));
        E[a][1] = (int)lround(sqrt(2.0) * sin(pi * (2 * a - 1) / 4.0));
    }
    WT[0] = 4.0 / 9.0;
    for (int a = 1; a <= 4; ++a) WT[a] = 1.0 / 9.0;
    for (int a = 5; a <= 8; ++a) WT[a] = 1.0 / 36.0;
    for (int a = 0; a < 9; ++a)
        for (int b = 0; b < 9; ++b)
            if (E[b][0] == -E[a][0] && E[b][1] == -E[a][1]) OPP[a] = b;
    lattice_ready = 1;
}

void orc_velocity_set(int32_t *ex, int32_t *ey, double *w, int32_t *opp)
{
    lattice_init();
    for (int a = 0; a < 9; ++a) {
        ex[a] = E[a][0]; ey[a] = E[a][1]; w[a] = WT[a]; opp[a] = OPP[a];
    }
}

static inline int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }
static inline size_t at(const orc_params *p, int x, int y)
{
    return (size_t)wrap(y, p->ny) * (size_t)p->nx + (size_t)wrap(x, p->nx);
}

/* eq. (3) */
void orc_equilibrium(double rho, double ux, double uy, double *feq)
{
    lattice_init();
    double uu = ux * ux + uy * uy;
    for (int a = 0; a < 9; ++a) {
        double eu = E[a][0] * ux + E[a][1] * uy;
        feq[a] = WT[a] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
    }
}

/* Threads of the per-node loops (OpenMP builds): n > 0 sets the count; returns
 * the count the next parallel loop uses (1 without OpenMP).  Every loop
 * writes only its own node, so results do not depend on the count. */
int orc_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* pseudopotential phi(rho) */
double orc_phi(double rho0, double rho) { return rho0 * (1.0 - exp(-rho / rho0)); }

/* --------------------------------------------------------------- geometry */
/* Electric layer and electrode side of every node (see the header). */
void orc_electric_layer(const orc_params *p, const uint8_t *solid, uint8_t *layer, uint8_t *top)
{
    int k = p->elec_layers;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t i = at(p, x, y);
            int is_top = (y >= p->ny / 2);
            top[i] = (uint8_t)(solid[i] ? 0 : is_top);
            layer[i] = 0;
            if (solid[i] || k <= 0) continue;
            uint32_t wall_bit = is_top ? 2u : 1u;
            if (!(p->elec_walls & wall_bit)) continue;
            int near = 0;
            for (int dy = -k; dy <= k && !near; ++dy)
                for (int dx = -k; dx <= k; ++dx)
                    if (solid[at(p, x + dx, y + dy)]) { near = 1; break; }
            layer[i] = (uint8_t)near;
        }
}

/*
 * Direction of the electric force on every node with elec_normal = 1 (see the
 * header): code[i] = alpha in 1..8 with n = e_alpha / |e_alpha|, or 0 where the
 * electrode direction applies (not a layer node, v = 0, or elec_normal = 0).
 * Brute force over the Chebyshev ball of radius elec_layers.
 */
void orc_electric_normal(const orc_params *p, const uint8_t *solid, uint8_t *code)
{
    lattice_init();
    size_t n = (size_t)p->nx * p->ny;
    uint8_t *layer = calloc(n, 1), *top = calloc(n, 1);
    orc_electric_layer(p, solid, layer, top);
    int k = p->elec_layers;
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t i = at(p, x, y);
            code[i] = 0;
            if (!p->elec_normal || !layer[i]) continue;
            int dmin = k + 1;
            for (int dy = -k; dy <= k; ++dy)
                for (int dx = -k; dx <= k; ++dx) {
                    int d = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
                    if (solid[at(p, x + dx, y + dy)] && d < dmin) dmin = d;
                }
            long vx = 0, vy = 0;
            for (int dy = -dmin; dy <= dmin; ++dy)
                for (int dx = -dmin; dx <= dmin; ++dx) {
                    int d = abs(dx) > abs(dy) ? abs(dx) : abs(dy);
                    if (d == dmin && solid[at(p, x + dx, y + dy)]) { vx += dx; vy += dy; }
                }
            int sx = (vx > 0) - (vx < 0), sy = (vy > 0) - (vy < 0);
            for (int a = 1; a <= 8; ++a)
                if (E[a][0] == sx && E[a][1] == sy) code[i] = (uint8_t)a;
        }
    free(layer); free(top);
}

/*
 * Per-node flag word, the format the GPU library exports for byte-exact
 * comparison: bit (alpha-1) = S(x + e_alpha) for alpha = 1..8, bit 8 = S(x),
 * bit 9 = electric layer, bit 10 = top electrode side, bits 11-14 = the
 * direction code of orc_electric_normal.  A solid node is 0x100.
 */
void orc_flags(const orc_params *p, const uint8_t *solid, uint16_t *flags)
{
    lattice_init();
    size_t n = (size_t)p->nx * p->ny;
    uint8_t *layer = calloc(n, 1), *top = calloc(n, 1), *code = calloc(n, 1);
    orc_electric_layer(p, solid, layer, top);
    orc_electric_normal(p, solid, code);
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t i = at(p, x, y);
            if (solid[i]) { flags[i] = 0x100; continue; }
            uint16_t v = 0;
            for (int a = 1; a <= 8; ++a)
                if (solid[at(p, x + E[a][0], y + E[a][1])]) v |= (uint16_t)(1u << (a - 1));
            if (layer[i]) v |= 0x200;
            if (top[i]) v |= 0x400;
            v |= (uint16_t)(code[i] << 11);
            flags[i] = v;
        }
    free(layer); free(top); free(code);
}

/* ------------------------------------------------------------------ moments */
/* eq. (2): rho = sum f, rho u = sum f e.  Solid nodes get 0. */
void orc_moments(const orc_params *p, const uint8_t *solid, const double *f,
                 double *rho, double *ux, double *uy)
{
    lattice_init();
    size_t n = (size_t)p->nx * p->ny;
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) {
        if (solid[i]) { rho[i] = ux[i] = uy[i] = 0.0; continue; }
        double r = 0, jx = 0, jy = 0;
        for (int a = 0; a < 9; ++a) {
            double fa = f[(size_t)a * n + i];
            r += fa; jx += fa * E[a][0]; jy += fa * E[a][1];
        }
        rho[i] = r; ux[i] = jx / r; uy[i] = jy / r;
    }
}

/* ------------------------------------------------------------------- forces */
/*
 * From the density field: Fs = eq. (5) over fluid neighbours, Fw = eq. (6),
 * Fe = electric force on conductive layer nodes.  Each output is [2][ny][nx]
 * (x plane then y plane); solid nodes get 0.  Any output may be NULL.
 */
static void forces_on(const orc_params *p, const uint8_t *solid, const uint8_t *layer,
                      const uint8_t *top, const uint8_t *code, const double *rho, double *Fs, double *Fw,
                      double *Fe)
{
    size_t n = (size_t)p->nx * p->ny;
    double G[9], W[9];
    G[0] = W[0] = 0.0;
    for (int a = 1; a <= 4; ++a) { G[a] = p->g_axis; W[a] = p->w_axis; }
    for (int a = 5; a <= 8; ++a) { G[a] = p->g_diag; W[a] = p->w_diag; }

    double *phi = malloc(n * sizeof(double));
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < n; ++i) phi[i] = solid[i] ? 0.0 : orc_phi(p->rho0, rho[i]);

#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y)
        for (int x = 0; x < p->nx; ++x) {
            size_t i = at(p, x, y);
            double sx = 0, sy = 0, wx = 0, wy = 0, ex = 0, ey = 0;
            if (!solid[i]) {
                for (int a = 1; a <= 8; ++a) {
                    size_t j = at(p, x + E[a][0], y + E[a][1]);
                    if (solid[j]) {          /* eq. (6), S = 1 */
                        wx += W[a] * E[a][0];
                        wy += W[a] * E[a][1];
                    } else {                 /* eq. (5) */
                        sx += G[a] * phi[j] * E[a][0];
                        sy += G[a] * phi[j] * E[a][1];
                    }
                }
                sx *= -phi[i]; sy *= -phi[i];
                wx *= -phi[i]; wy *= -phi[i];
                if (layer[i] && rho[i] >= p->rho_c) {
                    int a = code[i];
                    if (a == 0) {
                        ey = top[i] ? p->f_elec : -p->f_elec;
                    } else {        /* f along e_a / |e_a| */
                        double len = (a <= 4) ? 1.0 : sqrt(2.0);
                        ex = p->f_elec * (E[a][0] / len);
                        ey = p->f_elec * (E[a][1] / len);
                    }
                }
            }
            if (Fs) { Fs[i] = sx; Fs[n + i] = sy; }
            if (Fw) { Fw[i] = wx; Fw[n + i] = wy; }
            if (Fe) { Fe[i] = ex; Fe[n + i] = ey; }
        }
    free(phi);
}

void orc_forces(const orc_params *p, const uint8_t *solid, const double *rho,
                double *Fs, double *Fw, double *Fe)
{
    lattice_init();
    size_t n = (size_t)p->nx * p->ny;
    uint8_t *layer = calloc(n, 1), *top = calloc(n, 1), *code = calloc(n, 1);
    orc_electric_layer(p, solid, layer, top);
    orc_electric_normal(p, solid, code);
    forces_on(p, solid, layer, top, code, rho, Fs, Fw, Fe);
    free(layer); free(top); free(code);
}

/* --------------------------------------------------------------------- init */
/* f_alpha(x, 0) = f_alpha^eq(rho_init, u_init) on fluid nodes, 0 on solids. */
void orc_init(const orc_params *p, const uint8_t *solid, const double *rho,
              const double *ux, const double *uy, double *f)
{
    lattice_init();
    size_t n = (size_t)p->nx * p->ny;
    double feq[9];
    for (size_t i = 0; i < n; ++i) {
        if (solid[i]) { for (int a = 0; a < 9; ++a) f[(size_t)a * n + i] = 0.0; continue; }
        orc_equilibrium(rho[i], ux ? ux[i] : 0.0, uy ? uy[i] : 0.0, feq);
        for (int a = 0; a < 9; ++a) f[(size_t)a * n + i] = feq[a];
    }
}

/* ------------------------------------------------------ TRT with Guo forcing */
/* omega- of the TRT operator from tau (omega+ = 1/tau) and Lambda. */
double orc_trt_omega_minus(double tau, double magic)
{
    return 1.0 / (magic / (tau - 0.5) + 0.5);
}

/*
 * Collision of node i (see the header): rho and u = j / rho from eq. (2), F
 * the total force.  Writes the nine post-collision populations to fs.
 */
static void collide_trt_guo(const orc_params *p, const double *f, double *fs, size_t n, size_t i,
                            double rho, double ux, double uy, double Fx, double Fy)
{
    const double wp = 1.0 / p->tau;
    const double wm = orc_trt_omega_minus(p->tau, p->trt_magic);
    /* velocity of the equilibrium and of the source: (j + F/2) / rho */
    const double vx = ux + 0.5 * Fx / rho, vy = uy + 0.5 * Fy / rho;
    double feq[9], S[9], neq[9];
    orc_equilibrium(rho, vx, vy, feq);
    for (int a = 0; a < 9; ++a) {
        const double eu = E[a][0] * vx + E[a][1] * vy;
        const double eF = E[a][0] * Fx + E[a][1] * Fy;
        const double uF = vx * Fx + vy * Fy;
        S[a] = WT[a] * (3.0 * (eF - uF) + 9.0 * eu * eF);
        neq[a] = f[(size_t)a * n + i] - feq[a];
    }
    for (int a = 0; a < 9; ++a) {
        const int b = OPP[a];
        const double np = 0.5 * (neq[a] + neq[b]), nm = 0.5 * (neq[a] - neq[b]);
        const double sp = 0.5 * (S[a] + S[b]), sm = 0.5 * (S[a] - S[b]);
        fs[(size_t)a * n + i] = f[(size_t)a * n + i] - wp * np - wm * nm
                                + (1.0 - 0.5 * wp) * sp + (1.0 - 0.5 * wm) * sm;
    }
}

/* ------------------------------------------------------ MRT with Guo forcing */
/* Rows of the moment matrix, from the velocities: 1, -4 + 3|e|^2,
 * 4 - 21/2 |e|^2 + 9/2 |e|^4, e_x, (-5 + 3|e|^2) e_x, e_y, (-5 + 3|e|^2) e_y,
 * e_x^2 - e_y^2, e_x e_y; the rows are orthogonal, so M^-1 = M^T diag(1/|row|^2). */
static double MRT_M[9][9], MRT_N[9];
static int mrt_ready = 0;

static void mrt_init(void)
{
    if (mrt_ready) return;
    for (int a = 0; a < 9; ++a) {
        const double ex = E[a][0], ey = E[a][1], e2 = ex * ex + ey * ey;
        const double row[9] = {1.0, -4.0 + 3.0 * e2, 4.0 - 10.5 * e2 + 4.5 * e2 * e2, ex, (-5.0 + 3.0 * e2) * ex,
                               ey, (-5.0 + 3.0 * e2) * ey, ex * ex - ey * ey, ex * ey};
        for (int k = 0; k < 9; ++k) MRT_M[k][a] = row[k];
    }
    for (int k = 0; k < 9; ++k) {
        MRT_N[k] = 0.0;
        for (int a = 0; a < 9; ++a) MRT_N[k] += MRT_M[k][a] * MRT_M[k][a];
    }
    mrt_ready = 1;
}

/* Collision of node i with the MRT operator (see the header). */
static void collide_mrt_guo(const orc_params *p, const double *f, double *fs, size_t n, size_t i,
                            double rho, double ux, double uy, double Fx, double Fy)
{
    const double sq = orc_trt_omega_minus(p->tau, p->trt_magic), sn = 1.0 / p->tau;
    const double s[9] = {0.0, p->mrt_s_e, p->mrt_s_eps, 0.0, sq, 0.0, sq, sn, sn};
    const double vx = ux + 0.5 * Fx / rho, vy = uy + 0.5 * Fy / rho;
    double feq[9], S[9], ms[9];
    orc_equilibrium(rho, vx, vy, feq);
    for (int a = 0; a < 9; ++a) {
        const double eu = E[a][0] * vx + E[a][1] * vy;
        const double eF = E[a][0] * Fx + E[a][1] * Fy;
        const double uF = vx * Fx + vy * Fy;
        S[a] = WT[a] * (3.0 * (eF - uF) + 9.0 * eu * eF);
    }
    for (int k = 0; k < 9; ++k) {
        double m = 0.0, meq = 0.0, sf = 0.0;
        for (int a = 0; a < 9; ++a) {
            m += MRT_M[k][a] * f[(size_t)a * n + i];
            meq += MRT_M[k][a] * feq[a];
            sf += MRT_M[k][a] * S[a];
        }
        ms[k] = m - s[k] * (m - meq) + (1.0 - 0.5 * s[k]) * sf;
    }
    for (int a = 0; a < 9; ++a) {
        double v = 0.0;
        for (int k = 0; k < 9; ++k) v += MRT_M[k][a] * ms[k] / MRT_N[k];
        fs[(size_t)a * n + i] = v;
    }
}

/* --------------------------------------------------------------------- step */
/*
 * Advance nsteps time steps in place.  f holds the populations after
 * streaming (the state at time t).  One step:
 *   1. rho, u from eq. (2);
 *   2. forces Fs (5), Fw (6), electric f n, body rho g;
 *   3. u' from eq. (10);
 *   4. collision f* = f - (f - f^eq(rho, u'))/tau (right side of eq. (1));
 *      (collision = 1 or 2: steps 3-4 are the TRT or MRT collision with Guo
 *      forcing);
 *   5. streaming f(x + e, t + 1) = f*(x) (left side of eq. (1)), with a
 *      population arriving from a solid node replaced by bounce-back.
 * Returns 0, or 1 if a fluid density became non-positive or not finite.
 */
int orc_step_ext(const orc_params *p, const uint8_t *solid, double *f, int64_t nsteps, const double *acc);

int orc_step(const orc_params *p, const uint8_t *solid, double *f, int64_t nsteps)
{
    return orc_step_ext(p, solid, f, nsteps, NULL);
}

/* orc_step with a per-node acceleration field acc [2][ny][nx] (x plane, then
 * y plane; NULL for none) added to the driving acceleration: the body force
 * on node x is rho (g + acc(x)).  It carries forces the paper applies to the
 * fluid's mass in a prescribed pattern, like the artificial attraction that
 * gathers the fluid of its droplet run into one droplet. */
int orc_step_ext(const orc_params *p, const uint8_t *solid, double *f, int64_t nsteps, const double *acc)
{
    lattice_init();
    mrt_init();
    size_t n = (size_t)p->nx * p->ny;
    double *rho = malloc(n * sizeof(double)), *ux = malloc(n * sizeof(double)),
           *uy = malloc(n * sizeof(double));
    double *Fs = malloc(2 * n * sizeof(double)), *Fw = malloc(2 * n * sizeof(double)),
           *Fe = malloc(2 * n * sizeof(double));
    double *fs = malloc(9 * n * sizeof(double));
    uint8_t *layer = calloc(n, 1), *top = calloc(n, 1), *code = calloc(n, 1);
    orc_electric_layer(p, solid, layer, top);
    orc_electric_normal(p, solid, code);
    int bad = 0;

    for (int64_t t = 0; t < nsteps && !bad; ++t) {
        orc_moments(p, solid, f, rho, ux, uy);
#pragma omp parallel for schedule(static) reduction(| : bad)
        for (size_t i = 0; i < n; ++i)
            if (!solid[i] && !(rho[i] > 0.0 && isfinite(rho[i]))) bad = 1;
        if (bad) break;
        forces_on(p, solid, layer, top, code, rho, Fs, Fw, Fe);

        /* collision */
#pragma omp parallel for schedule(static)
        for (size_t i = 0; i < n; ++i) {
            double feq[9];
            if (solid[i]) { for (int a = 0; a < 9; ++a) fs[(size_t)a * n + i] = 0.0; continue; }
            double gx = p->accel_x, gy = p->accel_y;
            if (acc) { gx += acc[i]; gy += acc[n + i]; }
            double Fx = Fs[i] + Fw[i] + Fe[i] + rho[i] * gx;
            double Fy = Fs[n + i] + Fw[n + i] + Fe[n + i] + rho[i] * gy;
            if (p->collision == 1) {
                collide_trt_guo(p, f, fs, n, i, rho[i], ux[i], uy[i], Fx, Fy);
                continue;
            }
            if (p->collision == 2) {
                collide_mrt_guo(p, f, fs, n, i, rho[i], ux[i], uy[i], Fx, Fy);
                continue;
            }
            double upx = (rho[i] * ux[i] + p->tau * Fx) / rho[i];  /* eq. (10) */
            double upy = (rho[i] * uy[i] + p->tau * Fy) / rho[i];
            orc_equilibrium(rho[i], upx, upy, feq);
            for (int a = 0; a < 9; ++a) {
                double fa = f[(size_t)a * n + i];
                fs[(size_t)a * n + i] = fa - (fa - feq[a]) / p->tau;
            }
        }

        /* streaming with halfway bounce-back */
#pragma omp parallel for schedule(static)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                size_t i = at(p, x, y);
                if (solid[i]) continue;
                for (int a = 0; a < 9; ++a) {
                    size_t src = at(p, x - E[a][0], y - E[a][1]);
                    f[(size_t)a * n + i] = solid[src] ? fs[(size_t)OPP[a] * n + i]
                                                      : fs[(size_t)a * n + src];
                }
            }
    }
    free(rho); free(ux); free(uy); free(Fs); free(Fw); free(Fe); free(fs);
    free(layer); free(top); free(code);
    return bad;
}

/* ------------------------------------------------------------------- outputs */
/* Channel-averaged velocity profile (the paper's velocity figure): out[y] =
 * (1/nx) sum over the fluid nodes of row y of u_x from eq. (2), so that the
 * flux of eq. (11) is the sum of out over the rows. */
void orc_profile(const orc_params *p, const uint8_t *solid, const double *f, double *out)
{
    size_t n = (size_t)p->nx * p->ny;
    double *rho = malloc(n * sizeof(double)), *ux = malloc(n * sizeof(double)),
           *uy = malloc(n * sizeof(double));
    orc_moments(p, solid, f, rho, ux, uy);
    for (int y = 0; y < p->ny; ++y) {
        double q = 0;
        for (int x = 0; x < p->nx; ++x) {
            size_t i = at(p, x, y);
            if (!solid[i]) q += ux[i];
        }
        out[y] = q / p->nx;
    }
    free(rho); free(ux); free(uy);
}

/* eq. (11) with L = nx: Q = (1/nx) sum over fluid nodes of u_x; M = sum rho. */
void orc_flux(const orc_params *p, const uint8_t *solid, const double *f, double *Q, double *M)
{
    size_t n = (size_t)p->nx * p->ny;
    double *rho = malloc(n * sizeof(double)), *ux = malloc(n * sizeof(double)),
           *uy = malloc(n * sizeof(double));
    orc_moments(p, solid, f, rho, ux, uy);
    double q = 0, m = 0;
    for (size_t i = 0; i < n; ++i)
        if (!solid[i]) { q += ux[i]; m += rho[i]; }
    *Q = q / p->nx;
    *M = m;
    free(rho); free(ux); free(uy);
}
