"""Pins of the contact-angle measurement (paper_0708_4182_amd/measure.py) on synthetic
droplets of known angle (CPU only).

A tanh droplet profile rho(r) = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2(r - R)/W)
centred at (x_c, y_c) has its rho = level contour on the circle of radius
R_c = R + (W/2) artanh(((rho_l + rho_v)/2 - level) / ((rho_l - rho_v)/2)) about the
same centre, so the angle it makes with the wall plane y_w is exactly
arccos((y_w - y_c) / R_c).  Caps below, at and above 90 degrees pin the sign
and the offset of cos(theta) = (y_w - y_c)/R and the wall plane y_w = 0.5.
"""
import numpy as np
import pytest

from paper_0708_4182_amd.measure import base_angle, contact_angle
from paper_0708_4182_amd import inputs as I

RL, RV, W = 2.0, 0.15, 2.0
NX, NY = 160, 72


def cap(theta_deg, R=24.0, y_wall=0.5):
    th = np.radians(theta_deg)
    yc = y_wall - R * np.cos(th)
    solid = I.flat_channel(NX, NY)
    rho = I.droplet_density(NX, NY, R, RL, RV, width=W, cx=(NX - 1) / 2 + 0.3, cy=yc)
    rho = np.where(solid == 0, rho, 0.0)
    Rc = R + W / 2 * np.arctanh(((RL + RV) / 2 - 1.0) / ((RL - RV) / 2))
    exact = np.degrees(np.arccos((y_wall - yc) / Rc))
    return rho, solid == 0, exact, (yc, Rc)


@pytest.mark.parametrize("theta", [45.0, 60.0, 90.0, 120.0, 135.0, 150.0])
def test_contact_angle_of_synthetic_caps(theta):
    rho, fluid, exact, (yc, Rc) = cap(theta)
    got, (xcf, ycf, Rf) = contact_angle(rho, fluid, y_max=NY - 8)
    assert abs(np.degrees(got) - exact) < 0.2, (np.degrees(got), exact)
    assert abs(ycf - yc) < 0.15 and abs(Rf - Rc) < 0.15
    assert abs(xcf - ((NX - 1) / 2 + 0.3)) < 0.05


def test_contact_angle_changes_with_the_wall_plane():
    """Moving the wall plane by dy moves cos(theta) by dy / R."""
    rho, fluid, _, (yc, Rc) = cap(120.0)
    a0 = np.cos(contact_angle(rho, fluid, y_max=NY - 8)[0])
    a1 = np.cos(contact_angle(rho, fluid, y_max=NY - 8, y_wall=1.5)[0])
    assert abs((a1 - a0) - 1.0 / Rc) < 2e-3


def test_base_angle_cross_check():
    """The base-width / apex-height estimate agrees with the circle fit to a
    few degrees on resolved caps (it sees the lattice through whole nodes)."""
    for theta in (60.0, 90.0, 120.0):
        rho, fluid, exact, _ = cap(theta, R=30.0)
        assert abs(np.degrees(base_angle(rho)) - exact) < 6.0


def test_degenerate_fit_raises():
    """A cap lower than the dropped near-wall band leaves no contour to fit."""
    rho, fluid, _, _ = cap(30.0, R=20.0)
    with pytest.raises(ValueError):
        contact_angle(rho, fluid, y_max=NY - 8)
    with pytest.raises(ValueError):
        contact_angle(np.full((NY, NX), 0.5), fluid)
