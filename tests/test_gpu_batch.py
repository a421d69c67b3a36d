"""GPU tests of the batched engine (lbm_batch_* through the C ABI).

The batch runs every channel with the same tile code as a single lattice, so a
channel inside the batch must be bitwise identical to the same channel run
alone; graph replays must be bitwise identical to eager launches; retiring a
channel freezes it.  Parity against the FP64 oracle uses the same 1e-5 bar as
the single-lattice tests.  The two- and three-step kernels (set_kernel) must
give bitwise the one-step results, eagerly, in graphs whose length is not a
multiple of the steps per launch, and after retiring channels.
"""
import numpy as np
import pytest

import oracle as O
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


def small_sweep(n=6, seed=3, storage=0, layers=2):
    """Sweep-table channels shrunk to test sizes (uneven shapes, own G and f)."""
    rng = I.SplitMix64(seed)
    cases = []
    for i in range(n):
        ny = rng.randint(20, 70)
        nx = rng.randint(40, 300)
        b = rng.randint(0, 4)
        G = -5.5 + rng.uniform()
        f = 3e-3 * rng.uniform()
        solid = I.periodic_bumps(nx, ny, 5, b, 16, seed * 100 + i)
        cases.append(I.channel_case(nx, ny, solid, G=G, f_elec=f, accel=2e-6, seed=seed * 100 + i,
                                    storage=storage, layers=layers, name=f"ch{i}"))
    return cases


def run_single(lbm, case, n):
    s = lbm.from_case(case)
    s.step(n)
    return s


@pytest.mark.parametrize("storage,persistent", [(0, False), (1, False), (0, True), (1, True)])
def test_channel_in_batch_is_bitwise_single(lbm, storage, persistent):
    cases = small_sweep(storage=storage)
    b = lbm.Batch(cases)
    b.set_schedule(persistent)
    b.step(60)
    for i, c in enumerate(cases):
        ref = run_single(lbm, c, 60).moments()
        for x, y in zip(b.moments(i), ref):
            np.testing.assert_array_equal(x, y)
        assert b.steps_done(i) == 60


def test_geometry_bit_exact(lbm):
    cases = small_sweep()
    b = lbm.Batch(cases)
    for i, c in enumerate(cases):
        np.testing.assert_array_equal(b.geometry(i), O.flags(c.params, c.solid))


@pytest.mark.parametrize("persistent", [False, True])
def test_graph_replays_equal_eager(lbm, persistent):
    cases = small_sweep(n=5, seed=7)
    eager = lbm.Batch(cases)
    graph = lbm.Batch(cases)
    graph.set_schedule(persistent)
    graph.set_graph(10)
    for rep in range(3):
        eager.step(10)
        graph.step(10)
        # eager work and synchronisation between replays
        Qe, Me = eager.flux()
        Qg, Mg = graph.flux()
        np.testing.assert_array_equal(Qe, Qg)
        np.testing.assert_array_equal(Me, Mg)
        for i in range(len(cases)):
            for x, y in zip(eager.moments(i), graph.moments(i)):
                np.testing.assert_array_equal(x, y)
    # an odd remainder runs eagerly after the replays
    eager.step(13)
    graph.step(13)
    for i in range(len(cases)):
        for x, y in zip(eager.moments(i), graph.moments(i)):
            np.testing.assert_array_equal(x, y)


def test_retire_freezes_channels(lbm):
    cases = small_sweep(n=5, seed=11)
    b = lbm.Batch(cases)
    b.set_graph(4)
    b.step(20)
    frozen = {i: b.moments(i) for i in (1, 3)}
    b.retire([0, 1, 0, 1, 0])
    b.step(21)
    for i in (1, 3):
        for x, y in zip(b.moments(i), frozen[i]):
            np.testing.assert_array_equal(x, y)
        assert b.steps_done(i) == 20
    for i in (0, 2, 4):
        ref = run_single(lbm, cases[i], 41).moments()
        for x, y in zip(b.moments(i), ref):
            np.testing.assert_array_equal(x, y)


def test_batch_flux_matches_single(lbm):
    cases = small_sweep(n=4, seed=5)
    b = lbm.Batch(cases)
    b.step(40)
    Q, M = b.flux()
    for i, c in enumerate(cases):
        q, m = run_single(lbm, c, 40).flux()
        assert abs(M[i] - m) <= 1e-12 * m
        assert abs(Q[i] - q) <= 1e-12 * max(abs(q), 1e-12)


def test_batch_parity_vs_oracle(lbm):
    from test_gpu_parity import conductivity_margin
    cases = small_sweep(n=3, seed=21)
    for c in cases:
        assert conductivity_margin(c, 200) > 1e-5
    b = lbm.Batch(cases)
    b.step(200)
    for i, c in enumerate(cases):
        rho, ux, uy = (a.astype(np.float64) for a in b.moments(i))
        f = O.run(c, 200)
        ro, uxo, uyo = O.moments(c.params, c.solid, f)
        fl = c.solid == 0
        er = np.abs(rho - ro)[fl].max() / ro[fl].max()
        eu = np.hypot(ux - uxo, uy - uyo)[fl].max() / np.hypot(uxo, uyo)[fl].max()
        print(f"channel {i} {c.params.nx}x{c.params.ny}: err_rho={er:.2e} err_u={eu:.2e}")
        assert er < 1e-5 and eu < 1e-5


def test_batch_autotune_keeps_state(lbm):
    cases = small_sweep(n=4, seed=9)
    b = lbm.Batch(cases)
    b.step(10)
    before = [b.moments(i) for i in range(len(cases))]
    bx, rows, us = b.autotune(reps=2)
    assert bx in (64, 128, 256, 512) and rows in (16, 32, 64) and us > 0
    assert b.kernel() in ("fused", "two", "three")
    print(f"batch autotune: {b.kernel()} block_x {bx} rows {rows}: {us:.1f} us/step")
    for i in range(len(cases)):
        for x, y in zip(b.moments(i), before[i]):
            np.testing.assert_array_equal(x, y)
    b.step(15)
    for i, c in enumerate(cases):
        for x, y in zip(b.moments(i), run_single(lbm, c, 25).moments()):
            np.testing.assert_array_equal(x, y)


def test_batch_set_forces_and_init_device(lbm):
    import torch
    cases = small_sweep(n=3, seed=13)
    b = lbm.Batch(cases)
    b.set_forces(1, 2.5e-3, 3e-6)
    c1 = cases[1]
    c1.params = c1.params.replace(f_elec=2.5e-3, accel_x=3e-6)
    b.step(30)
    for x, y in zip(b.moments(1), run_single(lbm, c1, 30).moments()):
        np.testing.assert_array_equal(x, y)
    # warm start of channel 2 from device fields equals a fresh start
    rho = torch.tensor(cases[2].rho.astype(np.float32), device="cuda")
    b.init_device(2, rho)
    assert b.steps_done(2) == 0
    b.step(30)
    for x, y in zip(b.moments(2), run_single(lbm, cases[2], 30).moments()):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("kernel,storage,block_x", [("two", 0, 256), ("three", 0, 512), ("two", 1, 512),
                                                    ("three", 1, 256), ("two", 2, 256), ("three", 2, 512)])
def test_multi_step_batch_is_bitwise_single(lbm, kernel, storage, block_x):
    cases = small_sweep(storage=storage)
    b = lbm.Batch(cases)
    b.set_tile(block_x, 16)
    b.set_kernel(kernel)
    assert b.kernel() == kernel
    b.step(61)     # 61 = 20 x 3 + 1 = 30 x 2 + 1: the last step runs alone
    for i, c in enumerate(cases):
        ref = run_single(lbm, c, 61).moments()
        for x, y in zip(b.moments(i), ref):
            np.testing.assert_array_equal(x, y, err_msg=f"channel {i}")
        assert b.steps_done(i) == 61


@pytest.mark.parametrize("kernel,graph_steps", [("two", 2), ("two", 10), ("three", 4), ("three", 10)])
def test_multi_step_graph_equals_eager(lbm, kernel, graph_steps):
    """Replays of graphs of k-step launches plus single-step remainders (two
    steps under the two-step kernel is one launch: each replay flips the
    buffers) against eager one-step launches."""
    cases = small_sweep(n=5, seed=7)
    eager = lbm.Batch(cases)
    graph = lbm.Batch(cases)
    graph.set_kernel(kernel)
    graph.set_graph(graph_steps)
    for rep in range(3):
        eager.step(graph_steps)
        graph.step(graph_steps)
        Qe, Me = eager.flux()
        Qg, Mg = graph.flux()
        np.testing.assert_array_equal(Qe, Qg)
        np.testing.assert_array_equal(Me, Mg)
    eager.step(13)
    graph.step(13)
    for i in range(len(cases)):
        for x, y in zip(eager.moments(i), graph.moments(i)):
            np.testing.assert_array_equal(x, y)


def test_multi_step_retire(lbm):
    cases = small_sweep(n=5, seed=11)
    b = lbm.Batch(cases)
    b.set_kernel("three")
    b.step(20)
    frozen = {i: b.moments(i) for i in (0, 4)}
    b.retire([1, 0, 0, 0, 1])
    b.step(22)
    for i in (0, 4):
        for x, y in zip(b.moments(i), frozen[i]):
            np.testing.assert_array_equal(x, y)
    for i in (1, 2, 3):
        for x, y in zip(b.moments(i), run_single(lbm, cases[i], 42).moments()):
            np.testing.assert_array_equal(x, y)


def test_multi_step_rejects_other_kernels(lbm):
    b = lbm.Batch(small_sweep(n=2, seed=2))
    for k in (1, 2, 3, 4, 7, -1):
        assert b.lib.lbm_batch_set_kernel(b.h, k) == -1
    b.set_kernel("two")
    b.set_kernel("fused")
    assert b.kernel() == "fused"


def test_sweep_table_in_the_bench_configuration(lbm):
    """The 256-channel sweep table (82 M nodes) as bench.py times it: FP16
    storage with stochastic rounding, kernel (steps per launch), schedule and
    tile autotuned, hipGraphs of 12 steps; 24 steps.  On sampled channels (the
    smallest, the largest and two between): bitwise equal to the same channel
    run alone (single-lattice kernel, same rounding step counts), and, except
    the largest (~1 M nodes, to keep the oracle's share of the test short),
    against the FP64 oracle within twice the error of the format itself (the
    oracle rounded to FP16 to nearest after every step, against the unrounded
    oracle): for a value spread evenly between its two neighbours, stochastic
    rounding's mean squared error is 1/6 of a last place squared against 1/12
    for rounding to nearest, a ratio of sqrt(2) in the 2-norm (measured
    1.36-1.52)."""
    nsteps = 24
    cases = [I.sweep_case(r, storage=1, rounding=1) for r in I.sweep_table(256, 0)]
    b = lbm.Batch(cases)
    b.autotune(reps=3)
    b.set_graph(12)
    b.step(nsteps)
    kernel = b.kernel()
    sizes = np.array([c.params.nx * c.params.ny for c in cases])
    order = np.argsort(sizes, kind="stable")
    for i in (order[0], order[len(order) // 3], order[2 * len(order) // 3], order[-1]):
        c = cases[int(i)]
        got = b.moments(int(i))
        ref = lbm.from_case(c)
        ref.step(nsteps)
        for x, y in zip(got, ref.moments()):
            np.testing.assert_array_equal(x, y, err_msg=f"channel {i}")
        if i == order[-1]:
            continue
        p, s = c.params, c.solid
        f = O.init(p, s, c.rho, c.ux, c.uy)
        fr = O.round_storage(p, s, f.copy(), 1)
        for _ in range(nsteps):
            O.step(p, s, f, 1)
            O.step(p, s, fr, 1)
            O.round_storage(p, s, fr, 1)
        exact = O.moments(p, s, f)
        rounded = O.moments(p, s, fr)
        gpu = tuple(a.astype(np.float64) for a in got)
        fl = s == 0
        er = np.linalg.norm((gpu[0] - exact[0])[fl])
        eu = np.linalg.norm(np.hypot(gpu[1] - exact[1], gpu[2] - exact[2])[fl])
        fr_ = np.linalg.norm((rounded[0] - exact[0])[fl])
        fu_ = np.linalg.norm(np.hypot(rounded[1] - exact[1], rounded[2] - exact[2])[fl])
        print(f"channel {i} {p.nx}x{p.ny} ({kernel}): 2-norm error rho {er:.2e} u {eu:.2e}; "
              f"format's own (nearest) {fr_:.2e} / {fu_:.2e}")
        assert er <= 2 * fr_ and eu <= 2 * fu_
