"""GPU checks of the per-node acceleration field (lbm_set_accel_field) and of
the paper's droplet run under reading R29 (experiments.paper_droplet), against
the FP64 oracle through the C ABI.

  - a random acceleration field on the parity lattices: 1e-5 (the norms and
    the conductivity-margin guard of test_gpu_parity.py); a uniform field is
    the driving acceleration bit for bit; the kernels and calls that do not
    take a field refuse it;
  - the released droplet (made by the oracle) with the attraction on, then
    with the electric force on its single layer: 1e-5 over 300 steps each
    (PAPER_STEPS below: the FP32 floor of this flow).
    The gathering phase itself starts from a spinodal state (0.85 lies inside
    the spinodal), where a 1e-7 perturbation grows 500-fold in 50 steps, so
    FP32 and FP64 trajectories part there by more than 1e-5; it is checked
    through the droplet it leads to:
  - the whole run on the GPU against the whole run in the oracle: the same
    steady droplet (angle within 0.05 degree, the same conductive interval
    of the substrate layer) and the same cos(theta) - cos(theta_0) per field
    within 2e-3.
"""
import numpy as np
import pytest

import oracle as O
from paper_0708_4182_amd import inputs as I
from paper_0708_4182_amd import measure

from test_gpu_parity import CASES, conductivity_margin, errors

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0708_4182_amd import lbm as L
    L.load_library()
    return L


def random_field(shape, seed, amp=1e-4):
    rng = np.random.default_rng(seed)
    return rng.uniform(-amp, amp, (2,) + shape).astype(np.float32)


@pytest.mark.parametrize("name,nsteps", [("ragged37x19", 300), ("ragged130x67", 300), ("rough256x128", 500)])
def test_accel_field_parity(lbm, name, nsteps):
    import torch
    c = CASES[name]()
    acc = random_field(c.solid.shape, 7)
    acc[:, c.solid != 0] = 0.0
    f = O.init(c.params, c.solid, c.rho, c.ux, c.uy)
    O.step_ext(c.params, c.solid, f, nsteps, acc.astype(np.float64))
    sim = lbm.from_case(c)
    sim.set_accel_field(torch.from_numpy(acc).cuda())
    sim.step(nsteps)
    rho, ux, uy = (a.astype(np.float64) for a in sim.moments())
    er, eu, umax = errors(c, rho, ux, uy, f)
    print(f"acceleration field {name} N={nsteps}: err_rho={er:.2e} err_u={eu:.2e}")
    assert er < TOL and eu < TOL


def test_uniform_field_is_the_driving_acceleration(lbm):
    import torch
    c = CASES["ragged130x67"]()
    g = (2e-6, -1e-6)
    a = lbm.from_case(c.__class__(c.params.replace(accel_x=g[0], accel_y=g[1]), c.solid, c.rho))
    b = lbm.from_case(c.__class__(c.params.replace(accel_x=0.0, accel_y=0.0), c.solid, c.rho))
    acc = torch.empty((2,) + c.solid.shape, dtype=torch.float32, device="cuda")
    acc[0], acc[1] = g
    b.set_accel_field(acc)
    a.step(60)
    b.step(60)
    for x, y in zip(a.moments(), b.moments()):
        np.testing.assert_array_equal(x, y)
    b.set_accel_field(None)            # and removing it goes back to the plain step
    b.set_forces(c.params.f_elec, g[0], g[1])
    a.step(10)
    b.step(10)
    for x, y in zip(a.moments(), b.moments()):
        np.testing.assert_array_equal(x, y)


def test_accel_field_guards(lbm):
    import torch
    c = CASES["ragged37x19"]()
    acc = torch.zeros((2,) + c.solid.shape, dtype=torch.float32, device="cuda")
    s = lbm.from_case(c)
    s.set_accel_field(acc)
    with pytest.raises(lbm.LBMError):
        s.set_kernel("split")
    with pytest.raises(lbm.LBMError):
        s.autotune(reps=1)
    with pytest.raises(ValueError):
        s.set_accel_field(torch.zeros((2, 3, 3), dtype=torch.float32, device="cuda"))
    t = lbm.from_case(c.__class__(c.params.replace(collision=1), c.solid, c.rho))
    with pytest.raises(lbm.LBMError):
        t.set_accel_field(acc)
    s.set_accel_field(None)
    s.set_kernel("split")              # allowed again once the field is removed


@pytest.fixture(scope="module")
def released():
    """The paper's droplet run in the oracle: gathered (10,000 steps) and
    released (20,000 steps)."""
    c = I.paper_droplet_case(0)
    p, s = c.params, c.solid
    f = O.init(p, s, c.rho)
    O.step_ext(p, s, f, 10_000, I.attraction_field(p.nx, p.ny, 3e-4, s).astype(np.float64))
    O.step(p, s, f, 20_000)
    return c, f


# Steps of the FP32 parity check on the paper's droplet.  The released droplet
# carries |u| up to 0.30 (currents of the interface at density ratio 66): the
# FP32 run departs from the FP64 oracle by 4e-6 .. 6e-6 of max |u| within 100
# steps and then wanders between 3e-6 and 1.6e-5 without a trend (measured
# over 100 .. 2000 steps for the attraction, f = 0.06, f = 0.15 and no force).
# That floor is the format's, not a growing error, and whether step 1000 lands
# under 1e-5 is chance; 300 steps sit at 4.8e-6 .. 6.3e-6 in all four runs.
PAPER_STEPS = 300


def test_released_droplet_parity(lbm, released):
    """From the oracle's released droplet: PAPER_STEPS steps with the attraction
    on, then PAPER_STEPS steps of the electric force f = 0.15 on the single layer."""
    import torch
    c0, f0 = released
    p, s = c0.params, c0.solid
    rho, ux, uy = O.moments(p, s, f0)
    acc = I.attraction_field(p.nx, p.ny, 3e-4, s)
    for label, params, field in (("attraction", p, acc), ("field f = 0.15", p.replace(f_elec=0.15), None)):
        c = I.Case(params, s, rho, ux, uy)
        if params.f_elec:
            margin = conductivity_margin(c, PAPER_STEPS)
            assert margin > 1e-5, f"too close to the conductivity threshold ({margin:.1e})"
        f = O.init(params, s, rho, ux, uy)
        if field is not None:
            O.step_ext(params, s, f, PAPER_STEPS, field.astype(np.float64))
        else:
            O.step(params, s, f, PAPER_STEPS)
        sim = lbm.from_case(c)
        if field is not None:
            sim.set_accel_field(torch.from_numpy(field).cuda())
        sim.step(PAPER_STEPS)
        g = tuple(a.astype(np.float64) for a in sim.moments())
        er, eu, umax = errors(c, *g, f)
        print(f"paper droplet, {label}, {PAPER_STEPS} steps: err_rho={er:.2e} err_u={eu:.2e} (max|u| {umax:.2e})")
        assert er < TOL and eu < TOL


def test_paper_droplet_run_matches_the_oracle(lbm, released):
    from paper_0708_4182_amd import experiments
    fs = (0.0, 0.06, 0.15)
    out = experiments.paper_droplet(fs=",".join(str(v) for v in fs))
    c0, f0 = released
    p, s = c0.params, c0.solid
    r, _, _ = O.moments(p, s, f0)
    th0, _ = measure.contact_angle(r, s == 0, y_max=p.ny - 4)
    cond = np.nonzero(r[1] >= p.rho_c)[0]
    print(f"paper droplet: GPU theta0 {out['theta0_deg']:.3f}, oracle {np.degrees(th0):.3f}; "
          f"x1, x2 GPU {out['x1']}, {out['x2']}, oracle {cond[0]}, {cond[-1]}")
    assert abs(out["theta0_deg"] - np.degrees(th0)) < 0.05
    assert (out["x1"], out["x2"]) == (int(cond[0]), int(cond[-1]))
    for e in out["fig3"]:
        f = f0.copy()
        q = p.replace(f_elec=e["f"])
        O.step(q, s, f, 10_000)
        rr, _, _ = O.moments(q, s, f)
        d = np.cos(measure.contact_angle(rr, s == 0, y_max=p.ny - 4)[0]) - np.cos(th0)
        print(f"  f = {e['f']}: dcos GPU {e['dcos']:.5f}, oracle {d:.5f}")
        assert abs(e["dcos"] - d) < 2e-3
