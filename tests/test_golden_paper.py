"""Pins against values the paper prints (text fixtures under tests/golden/).

- d2q9_velocity_set.txt: the velocity set of the lattice definition and the
  weights of eq. (3).  The oracle's lattice, its opposite-direction table and
  the mass / momentum / stress moments of the weights must agree with it.
- paper_parameters.txt: the printed simulation parameters.  The workload
  generators keep rho0, rho_c and the fluid-wall to fluid-fluid strength
  ratio w / G of the paper (the strengths themselves are rescaled, reading R1).
"""
from fractions import Fraction
from pathlib import Path

import numpy as np

import oracle as O
from paper_0708_4182_amd import inputs as I

GOLDEN = Path(__file__).parent / "golden"


def read_rows(name):
    rows = []
    for line in (GOLDEN / name).read_text().splitlines():
        line = line.split("#", 1)[0].strip()
        if line:
            rows.append(line.split())
    return rows


def paper_lattice():
    rows = read_rows("d2q9_velocity_set.txt")
    assert [int(r[0]) for r in rows] == list(range(9))
    e = np.array([(int(r[1]), int(r[2])) for r in rows])
    w = [Fraction(r[3]) for r in rows]
    return e, w


def paper_parameters():
    return {r[0]: float(r[1]) for r in read_rows("paper_parameters.txt")}


def test_fixture_velocity_set_is_the_angle_formula():
    """The fixture's integers are the lattice definition's cos/sin formulas."""
    e, _ = paper_lattice()
    for a in range(1, 5):
        ang = np.pi * (a - 1) / 2
        np.testing.assert_allclose(e[a], [np.cos(ang), np.sin(ang)], atol=1e-15)
    for a in range(5, 9):
        ang = np.pi * (2 * a - 1) / 4
        np.testing.assert_allclose(e[a], np.sqrt(2) * np.array([np.cos(ang), np.sin(ang)]), atol=1e-15)


def test_fixture_weights_are_normalised_and_isotropic():
    """Exact rational moments of the eq. (3) weights: sum 1, first moment 0,
    second moment I/3 (what lets eq. (3) reproduce rho, rho u, rho/3 + rho u u)."""
    e, w = paper_lattice()
    assert sum(w) == 1
    for i in range(2):
        assert sum(wa * int(ea[i]) for wa, ea in zip(w, e)) == 0
        for j in range(2):
            m = sum(wa * int(ea[i]) * int(ea[j]) for wa, ea in zip(w, e))
            assert m == (Fraction(1, 3) if i == j else 0)


def test_oracle_lattice_matches_fixture():
    e, w = paper_lattice()
    oe, ow, opp = O.velocity_set()
    np.testing.assert_array_equal(oe, e)
    np.testing.assert_array_equal(ow, np.array([float(x) for x in w]))
    for a in range(9):
        np.testing.assert_array_equal(e[opp[a]], -e[a])


def test_workload_defaults_keep_paper_constants():
    P = paper_parameters()
    p = I.Params(nx=8, ny=8)
    assert p.rho0 == P["rho0"]
    assert p.rho_c == P["rho_c"]
    assert abs(I.WALL_TO_FLUID - P["w_fluid_wall"] / P["G_fluid_fluid"]) < 1e-15
    # the wall strengths of every G keep that ratio, axis and diagonal alike
    for G in (-4.5, -5.0, -5.5):
        q = I.params_for_G(8, 8, G)
        assert abs(q.w_axis / q.g_axis - P["w_fluid_wall"] / P["G_fluid_fluid"]) < 1e-12
        assert abs(q.w_diag / q.g_diag - P["w_fluid_wall"] / P["G_fluid_fluid"]) < 1e-12


def test_critical_density_separates_the_phases():
    """rho_c = 1.0 lies between the vapour and liquid densities of every
    interaction strength the workloads use, so the conductor test of the
    electric force picks the liquid."""
    P = paper_parameters()
    for G in (-4.5, -5.0, -5.5):
        rv, rl = I.coexistence(G)
        assert rv < P["rho_c"] < rl


def test_literal_normalisation_of_the_printed_parameters_diverges():
    """Reading R1: the printed strengths (G = -0.52 with 2G on the axes, w =
    -0.14 likewise, tau = 0.9, rho0 = 1) taken literally in eq. (4)/(6), from
    the printed homogeneous state rho = 0.85 (+-1e-3 noise) on the printed
    100 x 50 box with flat walls, drive the FP64 oracle to negative densities
    within a few steps; the workloads' normalisation G w_a with G = -5 from the
    same state separates into two phases and stays bounded."""
    import numpy as np
    import pytest
    P = paper_parameters()
    nx, ny = int(P["box_nx"]), int(P["box_ny"])
    G, w = P["G_fluid_fluid"], P["w_fluid_wall"]
    s = I.flat_channel(nx, ny)
    rho = P["rho_init"] + I.noise(0, (ny, nx), 1e-3)
    p = I.Params(nx=nx, ny=ny, tau=P["tau"], rho0=P["rho0"], g_axis=2 * G, g_diag=G, w_axis=2 * w,
                 w_diag=w, f_elec=0.0)
    f = O.init(p, s, rho)
    with pytest.raises(FloatingPointError):
        O.step(p, s, f, 50)
    q = I.params_for_G(nx, ny, -5.0, tau=P["tau"], rho0=P["rho0"])
    f = O.init(q, s, rho)
    O.step(q, s, f, 3000)
    r, _, _ = O.moments(q, s, f)
    fl = s == 0
    assert 0.1 < r[fl].min() < 0.3 and 1.7 < r[fl].max() < 2.1
