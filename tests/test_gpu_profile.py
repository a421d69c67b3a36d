"""GPU velocity profile (lbm_profile, lbm_batch_profile: the channel-averaged
u_x per row of the paper's velocity figure) against the FP64 oracle's
definition, summing to the GPU flux Q to FP64 rounding, repeatable bit for
bit, and equal in a batch to the channel alone.  Bar: a row average of u_x
cannot be further off than the worst node, and the FP32 field bar is
max|du| <= 1e-5 max|u| (the norm of the BGK parity tests), so
max|d profile| <= 1e-5 max|u| over fluid nodes."""
import numpy as np
import pytest

import oracle as O

from test_gpu_parity import CASES

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0708_4182_amd import lbm as L
    L.load_library()
    return L


@pytest.mark.parametrize("name,nsteps", [("rough256x128", 1000), ("ragged130x67", 300), ("droplet128x64", 500)])
def test_profile_matches_oracle(lbm, name, nsteps):
    c = CASES[name]()
    sim = lbm.from_case(c)
    sim.step(nsteps)
    prof = sim.profile()
    f = O.run(c, nsteps)
    ref = O.profile(c.params, c.solid, f)
    _, ux, uy = O.moments(c.params, c.solid, f)
    umax = np.hypot(ux, uy)[c.solid == 0].max()
    err = np.abs(prof - ref).max() / umax
    print(f"profile {name} N={nsteps}: max err {err:.2e} of max|u| {umax:.3e} "
          f"({np.abs(prof - ref).max() / np.abs(ref).max():.2e} of max|profile|)")
    assert err < 1e-5
    Q, _ = sim.flux()
    assert abs(prof.sum() - Q) <= 1e-12 * np.abs(prof).sum()
    assert np.array_equal(prof, sim.profile())


def test_batch_profile_equals_single(lbm):
    cases = [CASES[n]() for n in ("ragged37x19", "ragged130x67", "ragged300x5")]
    b = lbm.Batch(cases)
    b.step(40)
    for i, c in enumerate(cases):
        s = lbm.from_case(c)
        s.step(40)
        assert np.array_equal(b.profile(i), s.profile())
