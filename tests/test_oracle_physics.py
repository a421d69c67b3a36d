"""Pins of the oracle's full time step against invariants and textbook limits.

CPU only.  Each test names what fixes the expected value:
  - exact invariants of eqs. (1)-(3) (mass, momentum, rest state);
  - the body-force momentum balance of the velocity shift, eq. (10);
  - plane Poiseuille flow between halfway-bounce-back walls (parabola with
    curvature -g/nu, nu = (tau - 1/2)/3, and zero slip at tau = 1/2 + sqrt(3)/4,
    He, Zou, Luo & Dembo, J. Stat. Phys. 87, 115 (1997));
  - shear-wave decay at rate nu k^2;
  - the flat-interface coexistence densities from the mechanical-stability
    (psi-Maxwell) rule of the pseudopotential equation of state
    p = rho/3 + (G/6) psi^2 (Shan & Chen 1993/1994), computed here by quadrature;
  - the Laplace law for free droplets;
  - the linear Young-Lippmann relation cos(theta) - cos(theta_0) proportional to f
    that the paper uses as its own check (eq. (9), Fig. 3);
  - mirror, translation and 90-degree rotation covariance of the scheme.
"""
import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import fsolve

from paper_0708_4182_amd import measure
import oracle as O
from paper_0708_4182_amd import inputs as I

PAPER_E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1),
                    (1, 1), (-1, 1), (-1, -1), (1, -1)])


def total_momentum(f):
    return np.einsum("a,ayx->", PAPER_E[:, 0].astype(float), f), \
        np.einsum("a,ayx->", PAPER_E[:, 1].astype(float), f)


# ------------------------------------------------------------------ invariants
def test_rest_state_is_fixed_point():
    """Uniform density at rest, no walls: every force vanishes, f stays f^eq."""
    n = 16
    p = I.params_for_G(n, n, -5.0)
    solid = np.zeros((n, n), np.uint8)
    f = O.init(p, solid, np.full((n, n), 1.7))
    f0 = f.copy()
    O.step(p, solid, f, 50)
    np.testing.assert_allclose(f, f0, rtol=0, atol=2e-15)


@pytest.mark.parametrize("f_elec,accel", [(0.0, 0.0), (2e-3, 1e-6)])
def test_mass_conservation_rough_channel(f_elec, accel):
    """Bounce-back and BGK conserve mass exactly: |dM|/M < 1e-12 after 2000 steps."""
    c = I.rough_channel_case(nx=128, ny=48, f_elec=f_elec, accel=accel, seed=3)
    f = O.init(c.params, c.solid, c.rho)
    _, M0 = O.flux(c.params, c.solid, f)
    O.step(c.params, c.solid, f, 2000)
    _, M1 = O.flux(c.params, c.solid, f)
    assert abs(M1 - M0) / M0 < 1e-12


def test_momentum_conserved_without_walls():
    """Periodic box, no solids, no external force: sum F_sigma = 0 so the
    total momentum is conserved to round-off."""
    n = 24
    rng = np.random.default_rng(0)
    p = I.params_for_G(n, n, -5.0)
    solid = np.zeros((n, n), np.uint8)
    rho = rng.uniform(0.2, 1.9, (n, n))
    u = rng.uniform(-0.02, 0.02, (2, n, n))
    f = O.init(p, solid, rho, u[0], u[1])
    j0 = np.array(total_momentum(f))
    O.step(p, solid, f, 200)
    j1 = np.array(total_momentum(f))
    np.testing.assert_allclose(j1, j0, atol=1e-12)


def test_body_force_adds_exact_momentum():
    """Velocity shift with F = rho g: post-collision momentum is j + rho g, so
    the total momentum grows by exactly M g per step (any tau)."""
    n = 12
    for tau in (0.7, 1.0, 1.6):
        p = I.Params(nx=n, ny=n, tau=tau, g_axis=-0.3, g_diag=-0.07,
                     accel_x=3e-5, accel_y=-1e-5)
        solid = np.zeros((n, n), np.uint8)
        rng = np.random.default_rng(1)
        f = O.init(p, solid, rng.uniform(0.5, 1.5, (n, n)))
        M = f.sum()
        j0 = np.array(total_momentum(f))
        O.step(p, solid, f, 10)
        j1 = np.array(total_momentum(f))
        np.testing.assert_allclose(j1 - j0, 10 * M * np.array([3e-5, -1e-5]), rtol=1e-9, atol=1e-15)


# ------------------------------------------------------------------ Poiseuille
def poiseuille(tau, ny=34, nx=4, g=1e-6, steps=60000):
    p = I.Params(nx=nx, ny=ny, tau=tau, g_axis=0, g_diag=0, w_axis=0, w_diag=0, accel_x=g)
    s = I.flat_channel(nx, ny)
    f = O.init(p, s, np.ones((ny, nx)))
    O.step(p, s, f, steps)
    rho, ux, uy = O.moments(p, s, f)
    y = np.arange(1, ny - 1)
    nu = (tau - 0.5) / 3
    analytic = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)   # walls at 0.5 and ny - 1.5
    return p, s, f, ux[1:-1, 0], uy, analytic, nu, g


@pytest.mark.parametrize("tau", [0.8, 1.0, 0.5 + np.sqrt(3) / 4])
def test_poiseuille_curvature_is_minus_g_over_nu(tau):
    p, s, f, u, uy, analytic, nu, g = poiseuille(tau)
    d2 = nu * (u[2:] - 2 * u[1:-1] + u[:-2])
    np.testing.assert_allclose(d2, -g, rtol=1e-8)
    assert np.abs(uy).max() < 1e-10 * np.abs(u).max()
    # halfway bounce-back puts the wall planes at 0.5 and ny - 1.5 up to O(g) slip
    assert np.abs(u - analytic).max() / analytic.max() < 1e-3


def test_poiseuille_zero_slip_at_magic_tau():
    """At tau = 1/2 + sqrt(3)/4 the physical velocity u + g/2 is the exact
    parabola with walls at 0.5 and ny - 1.5."""
    p, s, f, u, uy, analytic, nu, g = poiseuille(0.5 + np.sqrt(3) / 4)
    v = u + g / 2
    np.testing.assert_allclose(v, analytic, rtol=1e-8, atol=1e-9 * analytic.max())


def test_poiseuille_flux_closed_form():
    """eq. (11) on the steady Poiseuille state: Q = sum_y u_x(y), the midpoint
    sum of the parabola, g H^3/(12 nu) + g H/(24 nu), up to the O(g) slip."""
    p, s, f, u, uy, analytic, nu, g = poiseuille(1.0)
    Q, M = O.flux(p, s, f)
    H = p.ny - 2
    assert abs(Q - u.sum()) < 1e-15
    ref = g * H ** 3 / (12 * nu) + g * H / (24 * nu)
    assert abs(Q - ref) / ref < 1e-3
    assert abs(M - H * p.nx) < 1e-9


@pytest.mark.parametrize("tau", [0.8, 1.0])
def test_shear_wave_decay_rate(tau):
    """u_x = U sin(k y) decays as exp(-nu k^2 t) (to O(k^2) relative)."""
    nx, ny = 4, 64
    k = 2 * np.pi / ny
    p = I.Params(nx=nx, ny=ny, tau=tau, g_axis=0, g_diag=0, w_axis=0, w_diag=0)
    s = np.zeros((ny, nx), np.uint8)
    y = np.arange(ny)
    ux = np.tile((1e-3 * np.sin(k * y))[:, None], (1, nx))
    f = O.init(p, s, np.ones((ny, nx)), ux, np.zeros_like(ux))
    amps = []
    for _ in range(2):
        O.step(p, s, f, 200)
        _, u, _ = O.moments(p, s, f)
        amps.append(2 / ny * (u[:, 0] * np.sin(k * y)).sum())
    rate = -np.log(amps[1] / amps[0]) / 200
    nu = (tau - 0.5) / 3
    assert abs(rate / (nu * k * k) - 1) < 5e-3


# ------------------------------------------------------------ two-phase physics
def maxwell_coexistence(G):
    """Mechanical-stability coexistence of p = rho/3 + (G/6) psi^2:
    p(rv) = p(rl) and int_rv^rl (p0 - p) psi'/psi^2 drho = 0."""
    psi = lambda r: 1 - np.exp(-r)
    p = lambda r: r / 3 + G / 6 * psi(r) ** 2

    def eqs(v):
        rv, rl = v
        p0 = p(rv)
        integral = quad(lambda r: (p0 - p(r)) * np.exp(-r) / psi(r) ** 2, rv, rl)[0]
        return [p(rl) - p0, integral]

    return fsolve(eqs, [0.1, 2.0], xtol=1e-12)


@pytest.mark.parametrize("G", [-4.5, -5.0, -5.5])
def test_flat_interface_coexistence(G):
    nx, ny = 4, 160
    p = I.params_for_G(nx, ny, G)
    s = np.zeros((ny, nx), np.uint8)
    rv, rl = maxwell_coexistence(G)
    y = np.arange(ny)[:, None] * np.ones((1, nx))
    rho = rv + (rl - rv) * 0.5 * (np.tanh((y - 40) / 2) - np.tanh((y - 120) / 2))
    f = O.init(p, s, rho)
    O.step(p, s, f, 15000)
    r, _, _ = O.moments(p, s, f)
    assert abs(r[80, 0] / rl - 1) < 0.02
    assert abs(r[0, 0] / rv - 1) < 0.02
    assert abs(r[80, 0] - r[80, 3]) < 1e-12


@pytest.mark.slow
def test_laplace_law():
    """Free droplets in a periodic box: dp = p_in - p_out is linear in 1/R
    with a near-zero intercept (2D Laplace law dp = sigma / R)."""
    G = -5.0
    n = 64
    rv, rl = I.coexistence(G)
    pts = []
    for R in (8, 11, 14, 17):
        p = I.params_for_G(n, n, G)
        s = np.zeros((n, n), np.uint8)
        rho = I.droplet_density(n, n, R, rl, rv, cx=(n - 1) / 2, cy=(n - 1) / 2)
        f = O.init(p, s, rho)
        O.step(p, s, f, 5000)
        r, _, _ = O.moments(p, s, f)
        press = lambda x: x / 3 + G / 6 * (1 - np.exp(-x)) ** 2
        rin, rout = r[n // 2, n // 2], r[0, 0]
        Reff = np.sqrt(((r - rout) / (rin - rout)).sum() / np.pi)
        pts.append((1 / Reff, press(rin) - press(rout)))
    a = np.array(pts)
    A = np.stack([a[:, 0], np.ones(len(a))], 1)
    (sigma, b), *_ = np.linalg.lstsq(A, a[:, 1], rcond=None)
    pred = A @ [sigma, b]
    r2 = 1 - ((a[:, 1] - pred) ** 2).sum() / ((a[:, 1] - a[:, 1].mean()) ** 2).sum()
    assert r2 > 0.999
    assert abs(b) < 0.03 * a[:, 1].max()
    assert 0.03 < sigma < 0.08


@pytest.mark.slow
def test_young_lippmann_linearity():
    """eq. (9): cos(theta) - cos(theta_0) grows in proportion to f.

    Droplet of radius 20 on the bottom electrode of a 128x64 box, f on liquid
    within 2 cells of the wall, f = 0 .. 1e-3 in 5 steps, 5000 steps each.
    The slope itself is not pinned: the paper's Fig. 3 values are unavailable.
    """
    fs = np.array([0.0, 2.5e-4, 5e-4, 7.5e-4, 1e-3])
    cos = []
    for fe in fs:
        c = I.droplet_case(f_elec=fe)
        f = O.run(c, 5000)
        r, _, _ = O.moments(c.params, c.solid, f)
        th, _ = measure.contact_angle(r, c.solid == 0, y_max=c.params.ny - 4)
        cos.append(np.cos(th))
    d = np.array(cos) - cos[0]
    A = np.stack([fs, np.ones_like(fs)], 1)
    (slope, b), *_ = np.linalg.lstsq(A, d, rcond=None)
    pred = A @ [slope, b]
    r2 = 1 - ((d - pred) ** 2).sum() / ((d - d.mean()) ** 2).sum()
    assert slope > 0          # the field makes the liquid wet the electrode
    assert r2 > 0.99
    assert abs(b) < 0.05 * d.max()


# ---------------------------------------------------------------- symmetries
MIRROR_X = [0, 3, 2, 1, 4, 6, 5, 8, 7]          # e_alpha -> (-ex, ey)
ROT90 = [0, 2, 3, 4, 1, 6, 7, 8, 5]              # e_alpha -> R e_alpha, R = +90 deg


def test_mirror_symmetry_of_droplet():
    """Droplet without noise is symmetric about x = (nx-1)/2 and stays so."""
    c = I.droplet_case(noise_amp=0.0)
    f = O.run(c, 1000)
    r, ux, uy = O.moments(c.params, c.solid, f)
    np.testing.assert_allclose(r, r[:, ::-1], atol=1e-13)
    np.testing.assert_allclose(ux, -ux[:, ::-1], atol=1e-13)
    np.testing.assert_allclose(uy, uy[:, ::-1], atol=1e-13)


def random_state(p, solid, seed):
    rng = np.random.default_rng(seed)
    n = solid.shape
    rho = rng.uniform(0.3, 1.8, n)
    u = rng.uniform(-0.03, 0.03, (2,) + n)
    f = O.init(p, solid, rho, u[0], u[1])
    f *= 1 + 0.01 * rng.standard_normal(f.shape)       # off-equilibrium parts
    f[:, solid == 1] = 0
    return f


def test_translation_covariance_is_bitwise():
    c = I.rough_channel_case(nx=64, ny=32, f_elec=2e-3, accel=1e-5, seed=2)
    p, s = c.params, c.solid
    f = random_state(p, s, 0)
    dx, dy = 13, 0            # y shift would move the electrode halves
    g = np.roll(f, (dy, dx), axis=(1, 2)).copy()
    O.step(p, s, f, 5)
    O.step(p, np.roll(s, (dy, dx), axis=(0, 1)), g, 5)
    np.testing.assert_array_equal(np.roll(f, (dy, dx), axis=(1, 2)), g)


def test_rotation_covariance():
    """Rotating the state by 90 degrees commutes with the step (no electric
    force, whose layer depends on the wall side, and no body force)."""
    n = 24
    rng = np.random.default_rng(4)
    s = (rng.random((n, n)) < 0.1).astype(np.uint8)
    p = I.params_for_G(n, n, -5.0, tau=0.9)
    f = random_state(p, s, 1)

    def rot(field):           # node (x, y) -> (-y mod n, x)
        out = np.empty_like(field)
        yy, xx = np.mgrid[0:n, 0:n]
        out[..., xx, (-yy) % n] = field[..., yy, xx]
        return out

    def rot_f(f):
        g = np.empty_like(f)
        for a in range(9):
            g[ROT90[a]] = rot(f[a])
        return g

    g = rot_f(f)
    O.step(p, s, f, 3)
    O.step(p, rot(s), g, 3)
    np.testing.assert_allclose(rot_f(f), g, atol=1e-14)


def test_velocity_profile_is_the_zero_slip_parabola():
    """The channel-averaged profile of a steady Poiseuille flow at
    tau = 1/2 + sqrt(3)/4 is the exact parabola (after the g/2 shift to the
    physical velocity), and its sum over the rows is the flux of eq. (11)."""
    p, s, f, u, uy, analytic, nu, g = poiseuille(0.5 + np.sqrt(3) / 4)
    prof = O.profile(p, s, f)
    assert prof[0] == 0 and prof[-1] == 0                 # solid rows
    np.testing.assert_allclose(prof[1:-1] + g / 2, analytic, rtol=1e-8, atol=1e-9 * analytic.max())
    Q, _ = O.flux(p, s, f)
    assert abs(prof.sum() - Q) <= 1e-14 * abs(Q)


def test_velocity_profile_rough_channel_sums_to_flux():
    c = I.rough_channel_case(nx=64, ny=40, f_elec=1e-3, accel=1e-6, seed=1)
    f = O.run(c, 300)
    prof = O.profile(c.params, c.solid, f)
    _, ux, _ = O.moments(c.params, c.solid, f)
    np.testing.assert_allclose(prof, ux.sum(1) / c.params.nx, rtol=1e-13, atol=1e-18)
    Q, _ = O.flux(c.params, c.solid, f)
    assert abs(prof.sum() - Q) <= 1e-13 * abs(Q)
