"""GPU checks of stochastic rounding of 16-bit storage (lbm_params.rounding = 1)
through the C ABI.

  - the rounding itself, value by value: one step from a saved FP16 (or BF16)
    state gives post-collision values p; the same state widened exactly to
    FP32 storage gives p without rounding.  Every stochastically rounded
    value must be one of the two 16-bit neighbours of p, nearest rounding
    must give the nearest one, and over the ~70,000 values of a 128 x 64
    droplet the fraction rounded up must match (p - lo) / (hi - lo) within
    five standard deviations, overall and per quarter of that fraction;
  - reproducibility: one call per step, hipGraph replays, the 8-wave kernel
    and the batch (both schedules) give bitwise the eager single-lattice
    result (the step count advances within a call, across calls and across
    replays), and a saved state continues exactly as the uninterrupted run;
  - only the fused kernels run it (LBM_EINVAL for the others).
"""
import numpy as np
import pytest

from paper_0708_4182_amd import inputs as I

from test_gpu_parity import CASES

pytestmark = pytest.mark.gpu

HEADER = 16
RHO_REF = 1.0


@pytest.fixture(scope="module")
def lbm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0708_4182_amd import lbm as L
    L.load_library()
    return L


def droplet(storage, rounding=0):
    c = I.droplet_case(f_elec=1e-3)
    c.params = c.params.replace(storage=storage, rounding=rounding, rho_ref=RHO_REF)
    return c


def planes(data: bytes, storage: int, c) -> np.ndarray:
    """Populations [9][ny][nx] as float32 from a saved state."""
    nx, ny = c.params.nx, c.params.ny
    pitch = -(-nx // 64) * 64
    body = np.frombuffer(data, np.uint8, offset=HEADER)
    if storage == 0:
        v = body.view(np.float32)
    elif storage == 1:
        v = body.view(np.float16).astype(np.float32)
    else:
        v = (body.view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    return v[:9 * pitch * ny].reshape(9, ny, pitch)[:, :, :nx]


def widen(data: bytes, storage: int) -> bytes:
    """A 16-bit state as an FP32 state (exact)."""
    body = np.frombuffer(data, np.uint8, offset=HEADER)
    if storage == 1:
        v = body.view(np.float16).astype(np.float32)
    else:
        v = (body.view(np.uint16).astype(np.uint32) << 16).view(np.float32)
    return data[:HEADER] + v.tobytes()


def neighbours(p: np.ndarray, storage: int):
    """The 16-bit values just below and above each float32 value (equal if exact)."""
    if storage == 1:
        h = p.astype(np.float16)
        lo = np.where(h.astype(np.float32) > p, np.nextafter(h, np.float16(-np.inf)), h).astype(np.float32)
        hi = np.where(h.astype(np.float32) < p, np.nextafter(h, np.float16(np.inf)), h).astype(np.float32)
        return lo, hi, h.astype(np.float32)
    u = p.view(np.uint32)
    t = (u & np.uint32(0xFFFF0000)).view(np.float32)            # towards zero
    away = ((u & np.uint32(0xFFFF0000)) + np.uint32(0x10000)).view(np.float32)
    exact = t == p
    other = np.where(exact, t, away)
    lo, hi = np.minimum(t, other), np.maximum(t, other)
    # nearest even, as the hardware conversion does it
    rb = u + np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))
    return lo, hi, (rb & np.uint32(0xFFFF0000)).view(np.float32)


@pytest.mark.parametrize("storage", [1, 2])
def test_rounding_value_by_value(lbm, storage):
    c_sr, c_rn, c32 = droplet(storage, 1), droplet(storage, 0), droplet(0)
    warm = lbm.from_case(c_rn)
    warm.step(400)                        # an interface, velocities, a spread of magnitudes
    state = warm.save_state()
    runs = {}
    for name, case, data in (("sr", c_sr, state), ("rn", c_rn, state), ("p", c32, widen(state, storage))):
        s = lbm.from_case(case)
        s.load_state(data)
        s.step(1)
        runs[name] = planes(s.save_state(), 0 if name == "p" else storage, case)
    fluid = (lbm.from_case(c32).geometry() & 0x100) == 0
    p, sr, rn = (runs[k][:, fluid].ravel() for k in ("p", "sr", "rn"))
    lo, hi, nearest = neighbours(p, storage)
    assert np.array_equal(rn, nearest), f"{int((rn != nearest).sum())} nearest-rounded values differ"
    inside = (sr == lo) | (sr == hi)
    assert inside.all(), f"{int((~inside).sum())} values outside their two neighbours"
    open_ = hi > lo
    t = ((p - lo) / np.where(open_, hi - lo, 1))[open_].astype(np.float64)
    up = (sr == hi)[open_].astype(np.float64)
    dev = up.sum() - t.sum()
    sd = np.sqrt((t * (1 - t)).sum())
    print(f"storage {storage}: {open_.sum()} inexact values, rounded up {up.mean():.4f} vs expected "
          f"{t.mean():.4f}, deviation {dev / sd:+.2f} sd; subnormal-range values "
          f"{int((np.abs(p) < 6.1e-5).sum()) if storage == 1 else 0}")
    assert abs(dev) < 5 * sd
    for q in range(4):
        sel = (t >= q / 4) & (t < (q + 1) / 4)
        d, s = up[sel].sum() - t[sel].sum(), np.sqrt((t[sel] * (1 - t[sel])).sum())
        assert abs(d) < 5 * s + 1, (q, d, s)
    # not the nearest rounding: a fair share of values leaves the nearest neighbour
    assert (sr != rn).mean() > 0.1


def test_reproducible_graph_kernel8(lbm):
    c = droplet(1, 1)
    a = lbm.from_case(c)
    a.step(61)
    ref = a.moments()
    b = lbm.from_case(c)
    for _ in range(61):                   # one call per step: the count advances across calls too
        b.step(1)
    g = lbm.from_case(c)
    g.set_graph(10)                       # six replays and one eager step
    g.step(61)
    k8 = lbm.from_case(c)
    k8.set_kernel("fused8")
    k8.step(61)
    k2 = lbm.from_case(c)
    k2.set_kernel("two")             # thirty two-step launches and one fused step
    k2.step(61)
    k2g = lbm.from_case(c)
    k2g.set_kernel("two")
    k2g.set_graph(10)                # five launches per replay: the parity flips at each replay
    k2g.step(61)
    k3 = lbm.from_case(c)
    k3.set_kernel("three")           # twenty three-step launches and one fused step
    k3.step(61)
    k3g = lbm.from_case(c)
    k3g.set_kernel("three")
    k3g.set_graph(10)                # three three-step launches and one fused step per replay
    k3g.step(61)
    for name, other in (("per-call", b), ("graph", g), ("fused8", k8), ("two", k2), ("two graph", k2g),
                        ("three", k3), ("three graph", k3g)):
        for x, y in zip(ref, other.moments()):
            np.testing.assert_array_equal(x, y, err_msg=name)
    rn = lbm.from_case(droplet(1, 0))
    rn.step(61)
    assert not np.array_equal(rn.moments()[0], ref[0])


def test_state_continues_the_count(lbm):
    c = droplet(2, 1)
    a = lbm.from_case(c)
    a.step(40)
    saved = a.save_state()
    a.step(40)
    b = lbm.from_case(c)
    b.load_state(saved)
    b.step(40)
    for x, y in zip(a.moments(), b.moments()):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("persistent,kernel", [(False, "fused"), (True, "fused"), (False, "two"),
                                               (True, "three")])
def test_batch_equals_single(lbm, persistent, kernel):
    """The batch continues the rounding step count like a single lattice, also
    when launches advance two or three steps (graph of 4 steps: 2 + 2 or 3 + 1)."""
    cases = []
    for name in ("ragged37x19", "ragged130x67", "ragged300x5"):
        c = CASES[name]()
        c.params = c.params.replace(storage=1, rounding=1)
        cases.append(c)
    b = lbm.Batch(cases)
    b.set_schedule(persistent)
    b.set_kernel(kernel)
    b.set_graph(4)
    b.step(31)
    for i, c in enumerate(cases):
        ref = lbm.from_case(c)
        ref.step(31)
        for x, y in zip(b.moments(i), ref.moments()):
            np.testing.assert_array_equal(x, y)


def test_other_kernels_rejected(lbm):
    s = lbm.from_case(droplet(1, 1))
    for k in ("split", "wide2", "wide4"):
        with pytest.raises(lbm.LBMError, match="EINVAL"):
            s.set_kernel(k)
    s.set_kernel("fused8")
    s.set_kernel("two")
    s.set_kernel("three")
    s.set_kernel("fused")


def sr_definition(v, r, storage):
    """Stochastic rounding written out with integer operations on the FP32
    word u of each value: the random bits (low 13 for FP16, 16 for BF16) are
    added below the result's last place and the word is truncated; for FP16
    results in the subnormal range (FP32 biased exponent e < 113) the dropped
    field is 113 - e bits longer and the random bits sit at its top.  Returns
    the 16-bit patterns (finite values only)."""
    u = v.view(np.uint32).astype(np.uint64)
    r = r.astype(np.uint64)
    if storage == 2:
        return (((u + (r & 0xFFFF)) & 0xFFFF0000) >> 16).astype(np.uint16)
    e = ((u >> 23) & 0xFF).astype(np.int64)
    sh = np.clip(113 - e, 0, 10).astype(np.uint64)
    mask = (np.uint64(0x2000) << sh) - np.uint64(1)
    w = ((u + ((r & 0x1FFF) << sh)) & ~mask & 0xFFFFFFFF).astype(np.uint32)
    return w.view(np.float32).astype(np.float16).view(np.uint16)


@pytest.mark.parametrize("storage", [1, 2])
def test_encoder_matches_its_definition(lbm, storage):
    """lbm_round_sr, the encoder of the step kernels' stochastic rounding (a
    gfx950 conversion instruction), against sr_definition bit by bit: every
    finite value for BF16; for FP16 every value of magnitude 2^-24 .. 2^15
    (below 2^-24 the result must be 0 or 2^-24 with the value's sign; the
    range of the stored deviations lies far below 2^15); Inf and NaN pass."""
    import torch
    rng = np.random.default_rng(7 + storage)
    n = 1 << 20
    mag = 10.0 ** rng.uniform(-12, 4.5 if storage == 2 else 4.3, n)
    v = (np.where(rng.random(n) < 0.5, -1.0, 1.0) * mag).astype(np.float32)
    v[:6] = [0.0, -0.0, np.inf, -np.inf, np.nan, 1.0]
    r = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    out = lbm.round_sr(torch.from_numpy(v).cuda(), torch.from_numpy(r.view(np.int32)).cuda(), storage)
    got = out.cpu().numpy().view(np.uint16)
    fin = np.isfinite(v)
    ref = sr_definition(v, r, storage)
    if storage == 2:
        sel = fin
        dec = (got.astype(np.uint32) << 16).view(np.float32)
    else:
        sel = fin & (np.abs(v) >= 2.0 ** -24)
        dec = got.view(np.float16).astype(np.float32)
        tiny = fin & (np.abs(v) < 2.0 ** -24)
        assert np.all((dec[tiny] == 0) | (np.abs(dec[tiny]) == np.float32(2.0 ** -24)))
        assert np.all(np.signbit(dec[tiny]) == np.signbit(v[tiny]))
    bad = int((got[sel] != ref[sel]).sum())
    print(f"storage {storage}: {int(sel.sum())} values compared, {bad} differ")
    assert bad == 0
    assert np.isposinf(dec[2]) and np.isneginf(dec[3]) and np.isnan(dec[4]) and dec[5] == 1.0
    assert np.signbit(dec[1]) and dec[0] == 0
