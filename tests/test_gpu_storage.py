"""Long-run error of each population storage against the FP64 oracle.

  - The 512 x 128 instance of the benchmark's random-step channel generator
    (seed 0, f = 1e-3, g = 1e-6) after 20,000 steps: density and velocity
    error (maximum norms over fluid nodes, relative to the oracle's maxima)
    and the relative error of the flux of eq. (11).
  - The 128 x 64 droplet (R = 20, f = 1e-3 on the bottom electrode) after
    20,000 steps: the contact angle from each storage against the oracle's.

Over 20,000 steps rounding differences are amplified by the two-phase
dynamics, so these are stated errors with generous bars, not a parity bar:
the 1e-5 FP32 parity is held over 300-1000 steps in test_gpu_parity.py.
"""
import numpy as np
import pytest

import oracle as O
from measure import contact_angle
from paper_0708_4182_amd import inputs as I

pytestmark = pytest.mark.gpu

STEPS = 20_000


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0708_4182_amd import lbm as L
    L.load_library()
    return L


@pytest.fixture(scope="module")
def channel_ref():
    c = I.random_channel_case(nx=512, ny=128, seed=0)
    f = O.run(c, STEPS)
    return c, O.moments(c.params, c.solid, f), O.flux(c.params, c.solid, f)[0]


@pytest.fixture(scope="module")
def droplet_ref():
    c = I.droplet_case(f_elec=1e-3)
    f = O.run(c, STEPS)
    rho = O.moments(c.params, c.solid, f)[0]
    return c, contact_angle(rho, c.solid == 0, y_max=c.params.ny - 8)[0]


@pytest.mark.parametrize("storage,bound", [(0, 1e-3), (1, 0.1), (2, None)])
def test_channel_error_after_20k_steps(lbm, channel_ref, storage, bound):
    """FP32 and FP16: bounded (measured 2e-5 / 4e-5 and 2e-2 / 5e-2).  BF16
    keeps 8 significant bits of a deviation, far too few for the slow
    velocity and interface modes; over 20,000 steps its fields drift tens of
    percent from the physics (measured: flux 34% off).  Stated, not bounded."""
    c, (ro, uxo, uyo), Qo = channel_ref
    c = I.random_channel_case(nx=512, ny=128, seed=0, storage=storage)
    s = lbm.from_case(c)
    s.step(STEPS)
    rho, ux, uy = (a.astype(np.float64) for a in s.moments())
    Q, _ = s.flux()
    fl = c.solid == 0
    er = np.abs(rho - ro)[fl].max() / np.abs(ro[fl]).max()
    eu = np.hypot(ux - uxo, uy - uyo)[fl].max() / np.hypot(uxo, uyo)[fl].max()
    eq = abs(Q / Qo - 1)
    print(f"storage {storage}: 512x128 random channel, {STEPS} steps: err_rho {er:.2e}, err_u {eu:.2e}, "
          f"flux {eq:.2e} (Q oracle {Qo:.6e})")
    assert np.isfinite([er, eu, eq]).all()
    if bound is not None:
        assert er < bound and eu < bound and eq < bound


@pytest.mark.parametrize("storage,bound_deg", [(0, 0.1), (1, 0.5), (2, None)])
def test_droplet_angle_after_20k_steps(lbm, droplet_ref, storage, bound_deg):
    """FP32 and FP16 hold the contact angle (measured 0.000 and 0.015 degrees
    off); with BF16 storage the droplet does not keep its shape (stated)."""
    c0, theta_o = droplet_ref
    c = I.droplet_case(f_elec=1e-3)
    c.params = c.params.replace(storage=storage)
    s = lbm.from_case(c)
    s.step(STEPS)
    rho = s.moments()[0].astype(np.float64)
    assert np.isfinite(rho).all()
    try:
        theta = contact_angle(rho, c.solid == 0, y_max=c.params.ny - 8)[0]
    except (ValueError, np.linalg.LinAlgError):
        theta = float("nan")
    d = np.degrees(theta - theta_o)
    print(f"storage {storage}: droplet angle {np.degrees(theta):.3f} deg, oracle {np.degrees(theta_o):.3f} deg, "
          f"difference {d:+.3f} deg")
    if bound_deg is not None:
        assert abs(d) < bound_deg
