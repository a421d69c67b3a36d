"""Pins of the oracle's 16-bit storage rounding (oracle.round_storage, the
definition of FP16 / BF16 deviation storage) on the CPU."""
import numpy as np
import pytest

import oracle as O
from paper_0708_4182_amd import inputs as I


def state(storage, seed=0):
    c = I.rough_channel_case(nx=48, ny=24, f_elec=1e-3, accel=1e-6, seed=seed)
    c.params = c.params.replace(storage=storage)
    f = O.run(c, 20)
    return c, f


@pytest.mark.parametrize("storage,bits", [(1, 11), (2, 8)])
def test_rounding_error_is_half_a_last_place(storage, bits):
    """|r(d) - d| <= 2^-bits |d| (half a last place of a bits-bit significand,
    relative), solid nodes untouched, and rounding twice changes nothing."""
    c, f = state(storage)
    p = c.params
    _, w, _ = O.velocity_set()
    off = (w * p.rho_ref)[:, None, None]
    g = O.round_storage(p, c.solid, f.copy(), storage)
    fl = c.solid == 0
    d, r = (f - off)[:, fl], (g - off)[:, fl]
    # FP16 subnormal range (below 2^-14): absolute half last place 2^-25
    tiny = (np.abs(d) < 2.0 ** -14) if storage == 1 else np.zeros(d.shape, bool)
    ok = np.abs(r - d) <= np.where(tiny, 2.0 ** -25, 2.0 ** -bits * np.abs(d))
    assert ok.all()
    assert (r != d).mean() > 0.9            # FP64 values are almost never representable
    np.testing.assert_array_equal(g[:, ~fl], f[:, ~fl])
    np.testing.assert_array_equal(O.round_storage(p, c.solid, g.copy(), storage), g)


def test_rounding_matches_library_conversions():
    """FP16 as numpy's correctly rounded float16 cast; BF16 as torch's
    float32 -> bfloat16 conversion where the deviation is a float32 value."""
    torch = pytest.importorskip("torch")
    c, f = state(2)
    p = c.params
    _, w, _ = O.velocity_set()
    off = (w * p.rho_ref)[:, None, None]
    fl = c.solid == 0
    d32 = (f - off).astype(np.float32).astype(np.float64)
    g = O.round_storage(p, c.solid, off + d32, 2)
    lib = torch.from_numpy(d32.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_allclose((g - off)[:, fl], lib[:, fl], rtol=0, atol=1e-15)
    g16 = O.round_storage(p.replace(storage=1), c.solid, off + d32, 1)
    lib16 = torch.from_numpy(d32.astype(np.float32)).to(torch.float16).to(torch.float64).numpy()
    np.testing.assert_allclose((g16 - off)[:, fl], lib16[:, fl], rtol=0, atol=1e-15)


def test_fp32_storage_is_the_identity_and_default_reference_is_rho0():
    c, f = state(0)
    g = O.round_storage(c.params, c.solid, f.copy(), 0)
    np.testing.assert_array_equal(g, f)
    p = c.params.replace(rho_ref=0.0, storage=1)
    _, w, _ = O.velocity_set()
    rest = np.broadcast_to((w * p.rho0)[:, None, None], f.shape).copy()
    np.testing.assert_array_equal(O.round_storage(p, c.solid, rest.copy(), 1), rest)   # d = 0 exactly
