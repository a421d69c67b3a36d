"""GPU checks of the electric force along the local face normal
(lbm_params.elec_normal = 1) against the FP64 oracle, through the C ABI.

  - flag words, including the direction codes in bits 11-14, bit-exact on
    rough and ragged lattices for layer depths 1-3;
  - FP32 fields within 1e-5 of the oracle on the rough-channel crop and the
    ragged lattices, with the conductivity-margin guard of the BGK cases.
    With the sideways force on the step faces, layer nodes of the crop cross
    rho_c after a few hundred steps (seed 5: margin 1.0e-4 up to step 500,
    below 1e-7 by step 600; seeds 0-8 all below 1e-5 by step 1000), so the
    crop runs 500 steps;
  - on flat walls the local normal is the electrode direction: the GPU run is
    bitwise the elec_normal = 0 run;
  - the other step kernels and the batch give bitwise the fused kernel's
    results.
"""
import numpy as np
import pytest

import oracle as O
from paper_0708_4182_amd import inputs as I

from test_gpu_parity import CASES, conductivity_margin, errors, tiny_rough

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


def normal_case(name):
    c = NCASES[name]()
    c.params = c.params.replace(elec_normal=1)
    return c


NCASES = {
    "rough256x128": lambda: I.rough_channel_case(nx=256, ny=128, f_elec=2e-3, accel=1e-6, seed=ROUGH_SEED,
                                                 layers=ROUGH_LAYERS),
    "ragged37x19": CASES["ragged37x19"],
    "ragged130x67": CASES["ragged130x67"],
    "ragged300x5": CASES["ragged300x5"],
}
ROUGH_SEED, ROUGH_LAYERS = 5, 1


@pytest.mark.parametrize("layers", [1, 2, 3])
def test_flags_with_normals_bit_exact(lbm, layers):
    for c in (I.rough_channel_case(nx=256, ny=128, f_elec=2e-3, seed=2, layers=layers),
              tiny_rough(37, 19, 1, f_elec=3e-3, layers=layers), tiny_rough(130, 67, 2, f_elec=1e-3, layers=layers)):
        c.params = c.params.replace(elec_normal=1)
        g = lbm.from_case(c).geometry()
        o = O.flags(c.params, c.solid)
        np.testing.assert_array_equal(g, o)
        assert ((g >> 11) & 15).any()


@pytest.mark.parametrize("name,nsteps", [("rough256x128", 500), ("ragged37x19", 300),
                                         ("ragged130x67", 300), ("ragged300x5", 300)])
def test_normal_fp32_parity(lbm, name, nsteps):
    c = normal_case(name)
    margin = conductivity_margin(c, nsteps)
    assert margin > 1e-5, f"case too close to the conductivity threshold ({margin:.1e})"
    sim = lbm.from_case(c)
    sim.step(nsteps)
    rho, ux, uy = (a.astype(np.float64) for a in sim.moments())
    f = O.run(c, nsteps)
    er, eu, umax = errors(c, rho, ux, uy, f)
    print(f"local normal {name} N={nsteps}: err_rho={er:.2e} err_u={eu:.2e} (margin {margin:.1e})")
    assert er < TOL and eu < TOL


def test_flat_walls_equal_electrode_direction(lbm):
    c = CASES["droplet128x64"]()
    a = lbm.from_case(c)
    c1 = CASES["droplet128x64"]()
    c1.params = c1.params.replace(elec_normal=1)
    b = lbm.from_case(c1)
    assert ((b.geometry() >> 11) & 15).any()
    a.step(300)
    b.step(300)
    for x, y in zip(a.moments(), b.moments()):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("kernel,tile", [("fused8", (256, 0)), ("wide2", (64, 0)), ("split", (128, 0)),
                                         ("two", (256, 0)), ("three", (512, 0))])
def test_normal_kernels_bitwise_equal_fused(lbm, kernel, tile):
    c = normal_case("ragged130x67")
    a = lbm.from_case(c)
    b = lbm.from_case(c)
    b.set_kernel(kernel)
    b.set_tile(*tile)
    a.step(60)
    b.step(60)
    for x, y in zip(a.moments(), b.moments()):
        np.testing.assert_array_equal(x, y)


def test_normal_batch_bitwise_single(lbm):
    cases = [normal_case(n) for n in ("ragged37x19", "ragged130x67", "ragged300x5")]
    b = lbm.Batch(cases)
    b.step(50)
    for i, c in enumerate(cases):
        ref = lbm.from_case(c)
        ref.step(50)
        for x, y in zip(b.moments(i), ref.moments()):
            np.testing.assert_array_equal(x, y)
