"""GPU test of lbm_flux_static, the allocation-free variant of lbm_flux
(through the C ABI): on two calls in a row, the second on a smaller lattice,
its flux and mass are bitwise those of lbm_flux on the same state, and a
repeat on the first lattice after the smaller one is unchanged (the static
array keeps the last call's contents, and nothing of them leaks into the
next result)."""
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


def test_flux_static_matches_flux(lbm):
    import torch
    big = I.rough_channel_case(nx=1024, ny=2048, f_elec=1e-3, accel=1e-6, seed=1)   # 1024 reduction workgroups
    small = I.rough_channel_case(nx=96, ny=37, f_elec=1e-3, accel=1e-6, seed=2)     # 37
    a = lbm.from_case(big)
    b = lbm.from_case(small)
    a.step(20)
    b.step(20)
    before = torch.cuda.memory_allocated()
    qa, ma = a.flux_static()
    qb, mb = b.flux_static()
    assert torch.cuda.memory_allocated() == before
    print(f"static: big Q={qa:.10e} M={ma:.10e}; small Q={qb:.10e} M={mb:.10e}")
    assert (qa, ma) == a.flux()
    assert (qb, mb) == b.flux()
    assert np.isfinite([qa, ma, qb, mb]).all() and ma > mb > 0
    # the big lattice again, after the smaller call left its partials behind
    assert a.flux_static() == (qa, ma)
    # and after more steps, still the same as the workspace variant
    a.step(7)
    assert a.flux_static() == a.flux()


def test_flux_static_reports_divergence(lbm):
    """A diverged state gives LBM_EDIVERGED through the static variant too."""
    n = 32
    p = I.params_for_G(n, n, -12.0, tau=0.52)
    case = I.Case(p, np.zeros((n, n), np.uint8), 1.0 + 0.5 * I.noise(7, (n, n), 1.0))
    sim = lbm.from_case(case)
    sim.step(400)
    with pytest.raises(lbm.Diverged):
        sim.flux_static()
