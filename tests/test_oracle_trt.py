"""Pins of the oracle's second collision operator: TRT with Guo forcing.

This operator is not in the paper; it replaces the velocity shift of eq. (10)
and the BGK collision of eq. (1) while keeping the paper's forces, lattice and
bounce-back walls.  CPU only.  What fixes each expected value:
  - Guo forcing adds exactly F of momentum per node and step
    (Guo, Zheng & Shi, Phys. Rev. E 65, 046308, 2002), and keeps mass;
  - with Lambda = 3/16, plane Poiseuille flow between halfway bounce-back
    walls is exact at the nodes for every tau (Ginzburg & d'Humieres,
    Phys. Rev. E 68, 066614, 2003; Ginzburg, Verhaeghe & d'Humieres 2008);
    with the BGK choice Lambda = (tau - 1/2)^2 it is not (a tau-dependent slip);
  - Lambda = (tau - 1/2)^2 makes omega- = omega+, where TRT is BGK with Guo
    forcing, checked against an independent numpy step (np.roll streaming);
  - the shear viscosity depends on tau only: a shear wave decays at nu k^2.
"""
import numpy as np
import pytest

import oracle as O
from paper_0708_4182_amd import inputs as I

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def momentum(f):
    return np.array([np.einsum("a,ayx->", E[:, 0].astype(float), f),
                     np.einsum("a,ayx->", E[:, 1].astype(float), f)])


def trt(nx, ny, **kw):
    kw.setdefault("collision", 1)
    return I.Params(nx=nx, ny=ny, **kw)


def test_omega_minus_from_magic():
    assert abs(O.trt_omega_minus(1.0, 3 / 16) - 1 / 0.875) < 1e-15
    for tau in (0.6, 0.9, 1.7):
        assert abs(O.trt_omega_minus(tau, (tau - 0.5) ** 2) - 1 / tau) < 1e-14


@pytest.mark.parametrize("magic", [3 / 16, 1 / 4, 0.05])
def test_guo_force_adds_exact_momentum(magic):
    """Two-phase periodic box (no walls) with a body force: sum F_sigma = 0 and
    Guo's source adds F per node, so the total momentum grows by exactly M g
    per step, and mass is unchanged."""
    n = 16
    rng = np.random.default_rng(2)
    g = np.array([2e-5, -7e-6])
    p = I.params_for_G(n, n, -5.0, collision=1, trt_magic=magic, tau=0.9, accel_x=g[0], accel_y=g[1])
    solid = np.zeros((n, n), np.uint8)
    f = O.init(p, solid, rng.uniform(0.3, 1.8, (n, n)))
    M0 = f.sum()
    j0 = momentum(f)
    O.step(p, solid, f, 20)
    np.testing.assert_allclose(momentum(f) - j0, 20 * M0 * g, rtol=1e-8, atol=1e-13)
    assert abs(f.sum() - M0) / M0 < 1e-13


def test_mass_conservation_with_walls_and_field():
    c = I.rough_channel_case(nx=96, ny=40, f_elec=2e-3, accel=1e-6, seed=3)
    c.params = c.params.replace(collision=1)
    f = O.init(c.params, c.solid, c.rho)
    _, M0 = O.flux(c.params, c.solid, f)
    O.step(c.params, c.solid, f, 1500)
    _, M1 = O.flux(c.params, c.solid, f)
    assert abs(M1 - M0) / M0 < 1e-12


def poiseuille_trt(tau, magic, ny=18, nx=4, g=1e-6):
    p = trt(nx, ny, tau=tau, trt_magic=magic, g_axis=0, g_diag=0, w_axis=0, w_diag=0, accel_x=g)
    s = I.flat_channel(nx, ny)
    f = O.init(p, s, np.ones((ny, nx)))
    nu = (tau - 0.5) / 3
    H = ny - 2
    steps = int(40 * H * H / (np.pi ** 2 * nu)) + 1000     # 40 e-folds of the slowest mode
    O.step(p, s, f, steps)
    _, ux, uy = O.moments(p, s, f)
    y = np.arange(1, ny - 1)
    v = ux[1:-1, 0] + g / 2                                   # (j + F/2) / rho, rho = 1
    exact = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)         # walls at 0.5 and ny - 1.5
    return v, exact, uy


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_poiseuille_exact_at_magic_three_sixteenths(tau):
    v, exact, uy = poiseuille_trt(tau, 3 / 16)
    np.testing.assert_allclose(v, exact, rtol=1e-9, atol=1e-9 * exact.max())
    assert np.abs(uy).max() < 1e-10 * exact.max()


def test_poiseuille_bgk_choice_slips():
    """The same flow with Lambda = (tau - 1/2)^2 (BGK) misses the parabola by a
    tau-dependent slip, so the exactness above is a property of Lambda."""
    v, exact, _ = poiseuille_trt(1.7, (1.7 - 0.5) ** 2)
    assert np.abs(v - exact).max() / exact.max() > 1e-3


def numpy_bgk_guo_step(f, tau, g):
    """One step of BGK with Guo forcing, force rho g, on a wall-free periodic
    lattice: an independent formulation (np.roll streaming)."""
    rho = f.sum(0)
    j = np.einsum("ad,ayx->dyx", E.astype(float), f)
    F = rho[None] * np.asarray(g)[:, None, None]
    u = (j + 0.5 * F) / rho
    eu = np.einsum("ad,dyx->ayx", E.astype(float), u)
    eF = np.einsum("ad,dyx->ayx", E.astype(float), F)
    uF = (u * F).sum(0)
    uu = (u * u).sum(0)
    feq = W[:, None, None] * rho[None] * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * uu[None])
    S = W[:, None, None] * (3 * (eF - uF[None]) + 9 * eu * eF)
    fs = f - (f - feq) / tau + (1 - 0.5 / tau) * S
    return np.stack([np.roll(np.roll(fs[a], E[a][0], axis=1), E[a][1], axis=0) for a in range(9)])


@pytest.mark.parametrize("tau", [0.7, 1.3])
def test_bgk_limit_matches_independent_step(tau):
    n = 6
    rng = np.random.default_rng(4)
    g = (3e-4, -2e-4)
    p = trt(n, n, tau=tau, trt_magic=(tau - 0.5) ** 2, g_axis=0, g_diag=0, w_axis=0, w_diag=0,
            accel_x=g[0], accel_y=g[1])
    solid = np.zeros((n, n), np.uint8)
    u = rng.uniform(-0.05, 0.05, (2, n, n))
    f = O.init(p, solid, rng.uniform(0.8, 1.2, (n, n)), u[0], u[1])
    ref = f.copy()
    for _ in range(5):
        ref = numpy_bgk_guo_step(ref, tau, g)
    O.step(p, solid, f, 5)
    np.testing.assert_allclose(f, ref, rtol=0, atol=1e-14)


@pytest.mark.parametrize("magic", [3 / 16, 1 / 4])
def test_shear_wave_decay_rate(magic):
    """u_x = U sin(k y) decays as exp(-nu k^2 t) with nu = (tau - 1/2)/3 set by
    omega+ alone."""
    nx, ny, tau = 4, 64, 0.8
    k = 2 * np.pi / ny
    p = trt(nx, ny, tau=tau, trt_magic=magic, g_axis=0, g_diag=0, w_axis=0, w_diag=0)
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
    assert abs(rate / ((tau - 0.5) / 3 * k * k) - 1) < 5e-3
