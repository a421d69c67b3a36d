"""Pins of the oracle's third collision operator: MRT with Guo forcing.

Not in the paper, like TRT: the multiple-relaxation-time collision of
Lallemand & Luo (Phys. Rev. E 61, 6546, 2000) in its orthogonal moment basis,
with Guo's forcing term taken to moment space.  CPU only.  What fixes each
expected value:
  - with s_e = s_eps = 1/tau every even non-conserved moment relaxes at
    omega+ and every odd one at omega-: the operator is TRT, an implementation
    in velocity space (test_oracle_trt.py pins it), to rounding;
  - Guo forcing adds exactly F of momentum per node and step and keeps mass;
  - the shear viscosity is (tau - 1/2)/3 whatever s_e and s_eps, and with
    Lambda = 3/16 plane Poiseuille flow between halfway bounce-back walls is
    exact at the nodes (the wall position depends on s_nu and s_q only);
  - the bulk viscosity is zeta = (1/s_e - 1/2)/3 (Lallemand & Luo, for
    c_s^2 = 1/3): a standing sound wave decays at (nu + zeta) k^2 / 2, set by
    s_e and not by s_eps.
"""
import numpy as np
import pytest

import oracle as O
from paper_0708_4182_amd import inputs as I

E = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)])


def momentum(f):
    return np.array([np.einsum("a,ayx->", E[:, 0].astype(float), f),
                     np.einsum("a,ayx->", E[:, 1].astype(float), f)])


@pytest.mark.parametrize("tau,magic", [(0.8, 3 / 16), (1.3, 0.25)])
def test_mrt_at_trt_rates_is_trt(tau, magic):
    """Rough channel with the Shan-Chen forces, the electric force and a body
    force: MRT with s_e = s_eps = 1/tau against TRT, 300 steps."""
    c = I.rough_channel_case(nx=64, ny=36, f_elec=2e-3, accel=1e-6, seed=4)
    p = c.params.replace(tau=tau, trt_magic=magic)
    a = O.init(p, c.solid, c.rho)
    b = a.copy()
    O.step(p.replace(collision=1), c.solid, a, 300)
    O.step(p.replace(collision=2, mrt_s_e=1 / tau, mrt_s_eps=1 / tau), c.solid, b, 300)
    assert np.abs(a - b).max() < 1e-12


def test_mrt_differs_from_trt_at_other_rates():
    """The same run with Lallemand & Luo's s_e, s_eps: a different operator
    (so the test above is not passing for an operator that ignores them)."""
    c = I.rough_channel_case(nx=64, ny=36, f_elec=2e-3, accel=1e-6, seed=4)
    a = O.init(c.params, c.solid, c.rho)
    b = a.copy()
    O.step(c.params.replace(collision=1), c.solid, a, 100)
    O.step(c.params.replace(collision=2), c.solid, b, 100)
    assert np.abs(a - b).max() > 1e-6


def test_guo_force_adds_exact_momentum():
    n = 16
    rng = np.random.default_rng(3)
    g = np.array([-1.5e-5, 8e-6])
    p = I.params_for_G(n, n, -5.0, collision=2, tau=0.9, accel_x=g[0], accel_y=g[1])
    solid = np.zeros((n, n), np.uint8)
    f = O.init(p, solid, rng.uniform(0.3, 1.8, (n, n)))
    M0 = f.sum()
    j0 = momentum(f)
    O.step(p, solid, f, 20)
    np.testing.assert_allclose(momentum(f) - j0, 20 * M0 * g, rtol=1e-8, atol=1e-13)
    assert abs(f.sum() - M0) / M0 < 1e-13


@pytest.mark.parametrize("tau", [0.6, 1.0, 1.7])
def test_poiseuille_exact_at_magic_three_sixteenths(tau):
    ny, nx, g = 18, 4, 1e-6
    p = I.Params(nx=nx, ny=ny, tau=tau, collision=2, trt_magic=3 / 16, g_axis=0, g_diag=0, w_axis=0, w_diag=0,
                 accel_x=g)
    s = I.flat_channel(nx, ny)
    f = O.init(p, s, np.ones((ny, nx)))
    nu = (tau - 0.5) / 3
    H = ny - 2
    O.step(p, s, f, int(40 * H * H / (np.pi ** 2 * nu)) + 1000)
    _, ux, uy = O.moments(p, s, f)
    y = np.arange(1, ny - 1)
    v = ux[1:-1, 0] + g / 2
    exact = g / (2 * nu) * (y - 0.5) * (ny - 1.5 - y)
    np.testing.assert_allclose(v, exact, rtol=1e-9, atol=1e-9 * exact.max())
    assert np.abs(uy).max() < 1e-10 * exact.max()


def sound_decay_rate(tau, s_e, s_eps, nx=64, steps=(400, 800)):
    """Standing wave rho = 1 + A cos(k x), u = 0, on a periodic strip: the
    amplitude of the density mode at the given times, through the envelope
    of |a(t)| (maxima of the oscillation near each time)."""
    k = 2 * np.pi / nx
    p = I.Params(nx=nx, ny=2, tau=tau, collision=2, mrt_s_e=s_e, mrt_s_eps=s_eps, g_axis=0, g_diag=0,
                 w_axis=0, w_diag=0)
    s = np.zeros((2, nx), np.uint8)
    x = np.arange(nx)
    f = O.init(p, s, np.tile(1 + 1e-4 * np.cos(k * x), (2, 1)))
    cs = 1 / np.sqrt(3)
    period = 2 * np.pi / (cs * k)
    amps, t = [], 0
    for target in steps:
        # step to the nearest half period of the acoustic oscillation
        nt = int(round(round(target / (period / 2)) * period / 2))
        O.step(p, s, f, nt - t)
        t = nt
        rho, _, _ = O.moments(p, s, f)
        amps.append((t, abs(2 / nx * ((rho[0] - 1) * np.cos(k * x)).sum())))
    (t0, a0), (t1, a1) = amps
    return -np.log(a1 / a0) / (t1 - t0), k


@pytest.mark.parametrize("s_e", [1.0, 1.6])
def test_sound_wave_decays_at_shear_plus_bulk_viscosity(s_e):
    tau = 0.8
    rate, k = sound_decay_rate(tau, s_e, 1.2)
    nu, zeta = (tau - 0.5) / 3, (1 / s_e - 0.5) / 3
    assert abs(rate / ((nu + zeta) * k * k / 2) - 1) < 5e-3


def test_sound_decay_does_not_depend_on_s_eps():
    r1, _ = sound_decay_rate(0.8, 1.4, 1.0)
    r2, _ = sound_decay_rate(0.8, 1.4, 1.8)
    assert abs(r1 / r2 - 1) < 1e-3
