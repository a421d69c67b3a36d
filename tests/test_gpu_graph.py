"""hipGraph replays of the single-lattice step (lbm_set_graph) against ordinary
launches: bitwise equal at every checkpoint, with eager work (moments, flux)
and synchronisations between replays, across buffer parities, and after the
graph is dropped by a change of forces or tile."""
import numpy as np
import pytest

from paper_0708_4182_amd import inputs as I

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


def same(a, b):
    for x, y in zip(a.moments(), b.moments()):
        np.testing.assert_array_equal(x, y)
    assert a.flux() == b.flux()
    assert a.steps_done == b.steps_done


@pytest.mark.parametrize("name,kernel", [("ragged130x67", "fused"), ("droplet128x64", "fused8"),
                                         ("ragged37x19", "split"), ("ragged130x67", "two"),
                                         ("droplet128x64", "three")])
def test_graph_replays_equal_launches(lbm, name, kernel):
    c = CASES[name]()
    a = lbm.from_case(c)
    b = lbm.from_case(c)
    for s in (a, b):
        s.set_kernel(kernel)
    b.set_graph(20)
    # 13 eager steps first, so replays also start from the other buffer parity
    for n in (13, 40, 57, 20, 3, 100):
        a.step(n)
        b.step(n)
        same(a, b)


def test_graph_dropped_by_forces_and_tile(lbm):
    c = CASES["ragged130x67"]()
    a = lbm.from_case(c)
    b = lbm.from_case(c)
    b.set_graph(10)
    a.step(30)
    b.step(30)
    for s in (a, b):
        s.set_forces(2.5e-3, 3e-6, 0.0)
    a.step(40)
    b.step(40)
    same(a, b)
    for s in (a, b):
        s.set_tile(64, 7)
    a.step(25)
    b.step(25)
    same(a, b)
    b.set_graph(0)
    a.step(11)
    b.step(11)
    same(a, b)


def test_graph_trt_operator(lbm):
    c = CASES["ragged37x19"]()
    c.params = c.params.replace(collision=1)
    a = lbm.from_case(c)
    b = lbm.from_case(c)
    b.set_graph(8)
    a.step(64)
    b.step(64)
    same(a, b)


def test_graph_invalid_counts(lbm):
    sim = lbm.from_case(CASES["ragged37x19"]())
    for bad in (1, 3, -2, 4098, 5000):
        with pytest.raises(lbm.LBMError):
            sim.set_graph(bad)
    sim.set_graph(0)
    sim.set_graph(4096)
    sim.step(5)
    assert sim.steps_done == 5
