"""GPU tests of the learned warm start.

The warm start must (a) fall back to the plain cold start, step for step,
when the network's prediction is unusable (small 64 x 32 channels), and (b)
after training on steady channels, reach the cold start's steady flux in fewer
lattice updates on held-out seeds.  Q_inf and the cold steady times come from
the plain lattice Boltzmann runs (the reference of every warm start)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

NX, NY = 64, 32


@pytest.fixture(scope="module")
def ws():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0708_4182_amd import lbm, warmstart
    lbm.load_library()
    return warmstart


def test_unusable_prediction_falls_back_to_cold_start(ws):
    from paper_0708_4182_amd import inputs as I
    from paper_0708_4182_amd import net
    # the comparison needs cold runs that settle (the steady rule); some seeds of
    # this small channel keep changing their flux by more than the rule allows,
    # so the first three seeds of six that settle are used
    cases = [I.warm_case(s, nx=NX, ny=NY) for s in range(100, 106)]
    data = ws.steady_states(cases, max_steps=100_000)
    settled = np.flatnonzero(data["cold"] > 0)
    assert settled.size >= 3, f"only {settled.size} of 6 cold runs settle"
    sel = settled[:3]
    m = net.Net(NY, NX, 4, chans=(8, 8, 8, 8))
    m.set_params(np.full(m.n_params, np.nan, np.float32))       # every prediction is NaN
    scales = ws.Scales(np.zeros(3), np.ones(3))
    stats, warm, _, _ = ws.warm_vs_cold(m, scales, [cases[i] for i in sel], data["Q"][sel],
                                     data["cold"][sel], max_steps=100_000)
    assert stats["used_prediction"] == 0
    np.testing.assert_array_equal(warm, data["cold"][sel])


def test_trained_warm_start_saves_lattice_updates(ws):
    """The warm-start channels themselves (256 x 64), a small training set
    (512 seeds, 20 epochs) and 32 held-out seeds: on the seeds where the warm
    start settles on the cold start's steady flux (the others, which settle on
    another steady branch, count as failures), it needs fewer lattice
    updates."""
    import torch
    from paper_0708_4182_amd import inputs as I
    from paper_0708_4182_amd import net
    train, test = 512, 32
    cases = [I.warm_case(s) for s in range(train + test)]
    data = ws.steady_states(cases, log=print)
    X, fluid = ws.features(cases)
    T = data["T"]
    scales = ws.Scales.fit(T[:train], fluid[:train])
    Tn = ((T - scales.mean.reshape(1, 3, 1, 1)) / scales.std.reshape(1, 3, 1, 1)).astype(np.float32)
    m = net.Net(64, 256, 32)
    m.set_params(net.he_init(net.layer_shapes(), 0))
    Xd, Td, Fd = (torch.from_numpy(a).cuda() for a in (X, Tn, fluid))
    losses = ws.train(m, Xd[:train], Td[:train], Fd[:train], epochs=20, batch=32, seed=0)
    print("loss", losses[0][1], "->", losses[-1][1])
    assert losses[-1][1] < 0.05 * losses[0][1]
    stats, warm, sur, q_end = ws.warm_vs_cold(m, scales, cases[train:], data["Q"][train:],
                                              data["cold"][train:], log=print)
    cold = data["cold"][train:]
    ok = (warm >= 0) & (cold >= 0)
    assert stats["used_prediction"] == test
    assert stats["warm_failures"] <= 0.4 * test
    assert stats["median_speedup"] >= 1.3
    assert warm[ok].sum() < cold[ok].sum()
