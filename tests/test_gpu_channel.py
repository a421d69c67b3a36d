"""GPU checks of the channel flux (eq. (11)) at steady state.

  - Poiseuille limit: a smooth single-phase channel (G = W = f = 0) carries
    the textbook flux Q = g H^3 / (12 nu), H the distance between the halfway
    walls, to 1e-3 relative.  The FP64 oracle gives it to 3e-11 at tau = 1;
    FP32 stops short by about 1.5e-4: the last correction per step of the
    slowest viscous mode falls below the rounding of the stored populations.
  - Flux against the electric force: in the rough channel of the paper's
    channel figures (steps a = 8, b = 4, p = 32; a 256 x 128 lattice, 8 whole
    periods) the flux after 300 000 steps from the seeded cold start is
    compared with the FP64 oracle's stored values
    (tests/golden/flux_trend_rough256x128.txt) for f = 0 .. 2e-3.
    As the paper reports, any field lowers the flux below Q0.  The trend is
    not monotone: the oracle itself has Q(1.5e-3) above Q(1e-3) by 4.8e-4 Q0
    (the paper also describes a flux that rises again under strong fields in
    a narrow channel), and the GPU must reproduce that ordering.
    FP32 holds this two-phase steady flux to a few 1e-4 of Q0 (measured
    0.4 - 2.3e-4), not 1e-5: at a steady state each node's rounding error
    repeats identically every step instead of averaging out, and the slowest
    viscous mode (~2500 steps per e-fold) integrates it, so the FP32 map
    settles about 6e-8 x 2500 ~ 1.5e-4 away from the FP64 one.  Every storage
    reference (raw, vapour, liquid) gives the same error, and other noise
    seeds or G x (1 +- 1e-6) move the FP32 flux by only 1e-5, so the gap is
    this arithmetic bias, not storage rounding or a different branch.
"""
import numpy as np
import pytest

from paper_0708_4182_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0708_4182_amd import lbm as L
    L.load_library()
    return L


def test_poiseuille_flux(lbm):
    nx, ny, g, tau = 16, 66, 1e-6, 1.0
    solid = I.flat_channel(nx, ny)
    p = I.Params(nx=nx, ny=ny, tau=tau, g_axis=0.0, g_diag=0.0, w_axis=0.0, w_diag=0.0, f_elec=0.0,
                 accel_x=g, rho_ref=1.0)
    c = I.Case(p, solid, np.ones((ny, nx)))
    s = lbm.from_case(c)
    s.step(60_000)                      # slowest mode: H^2 / (pi^2 nu) = 2490 steps per e-fold
    Q, M = s.flux()
    H = ny - 2.0
    nu = (tau - 0.5) / 3.0
    Q_exact = g * H ** 3 / (12.0 * nu)
    print(f"Poiseuille: Q = {Q:.6e}, g H^3 / (12 nu) = {Q_exact:.6e}, rel {Q / Q_exact - 1:+.2e}")
    assert abs(Q / Q_exact - 1) <= 1e-3


def read_flux_trend():
    from pathlib import Path
    rows = []
    for line in (Path(__file__).parent / "golden" / "flux_trend_rough256x128.txt").read_text().splitlines():
        line = line.split("#", 1)[0].strip()
        if line:
            rows.append([float(v) for v in line.split()])
    a = np.array(rows)
    return a[:, 0], a[:, 1], a[:, 2]


def test_flux_against_field_matches_oracle(lbm):
    fs, Q_orc, M_orc = read_flux_trend()
    cases = [I.rough_channel_case(nx=256, ny=128, f_elec=f, seed=0) for f in fs]
    b = lbm.Batch(cases)
    for _ in range(30):
        b.step(10_000)
    Q, M = b.flux()
    q, q_orc = Q / Q[0], Q_orc / Q_orc[0]
    print("Q/Q0 GPU   :", " ".join(f"{v:.6f}" for v in q))
    print("Q/Q0 oracle:", " ".join(f"{v:.6f}" for v in q_orc))
    err = np.abs(Q - Q_orc) / Q_orc[0]
    print("flux error / Q0:", " ".join(f"{v:.1e}" for v in err),
          "mass error:", f"{np.max(np.abs(M / M_orc - 1)):.1e}")
    # FP32 mass after 300 000 steps: measured within 1.4e-6 of the oracle's
    np.testing.assert_allclose(M, M_orc, rtol=5e-6)
    assert np.all(err <= 5e-4)
    assert np.all(q[1:] < 1) and np.all(q_orc[1:] < 1)
    assert np.array_equal(np.sign(np.diff(q)), np.sign(np.diff(q_orc)))
