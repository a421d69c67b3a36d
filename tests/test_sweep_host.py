"""Host logic of the steady-flux sweep driver (CPU only, a stand-in batch).

  - plain rule: a channel retires at the first check where its flux moved by
    at most rtol over one window (an exponential approach gives the check
    the closed form predicts);
  - averaged rule (16-bit storage with stochastic rounding): a flux that
    carries noise never passes the plain rule, but its window means settle;
    the reported flux is exactly the mean of the last window's records.
"""
import numpy as np

from paper_0708_4182_amd import sweep as SW

from test_warmstart_host import FakeBatch as _Fake


class FakeBatch(_Fake):
    shapes = None

    def __init__(self, funcs):
        super().__init__(funcs)
        self.shapes = [(64, 256)] * self.n


def test_plain_rule_exponential_approach():
    # Q(t) = 1 + 0.1 exp(-t/1000); |Q(t) - Q(t - 1000)| = 0.1 exp(-t/1000)(e - 1) <= 1e-6 Q(t)
    b = FakeBatch([lambda t: 1 + 0.1 * np.exp(-t / 1000.0), lambda t: 2.0 + np.sin(t / 300.0)])
    res = SW.run_to_steady(b, check_every=100, window=1000, rtol=1e-6, max_steps=30_000)
    t_exact = 1000 * np.log(0.1 * (np.e - 1) / 1e-6)          # 12,054 -> first check at 12,100
    assert res.converged[0] and res.steps[0] == 12_100 and 12_000 < t_exact < 12_100
    assert res.Q[0] == res.history[0][-1][1]
    assert not res.converged[1] and res.steps[1] == 30_000


def noisy(seed, amp):
    rng = np.random.default_rng(seed)
    table = rng.standard_normal(1000)
    return lambda t: 1 + 0.1 * np.exp(-t / 1000.0) + amp * table[(t // 100) % 1000]


def test_averaged_rule_on_a_noisy_flux():
    """A noisy flux passes the plain rule only by chance (two noisy records
    within rtol of each other); the window means settle once the transient is
    below the noise of one window."""
    f = noisy(1, 1e-5)
    avg = SW.run_to_steady(FakeBatch([f]), check_every=100, window=1000, rtol=1e-5, max_steps=40_000,
                           average=True)
    assert avg.converged[0]
    last = [q for _, q in avg.history[0][-10:]]
    assert avg.Q[0] == np.mean(last)
    # the window mean is within a few times the noise of one window (1e-5 / sqrt(10)) of the
    # limit, and the transient has decayed to the order of rtol when it stops
    assert abs(avg.Q[0] - 1) < 5e-5
    t = avg.steps[0]
    assert 0.1 * np.exp(-(t - 1000) / 1000.0) * (np.e - 1) < 1e-4
    # without noise the averaged rule stops when consecutive window means agree to rtol
    clean = SW.run_to_steady(FakeBatch([lambda t: 1 + 0.1 * np.exp(-t / 1000.0)]), check_every=100,
                             window=1000, rtol=1e-6, max_steps=40_000, average=True)
    h = np.array([q for _, q in clean.history[0]])
    new, old = h[-10:].mean(), h[-20:-10].mean()
    assert clean.converged[0] and abs(new - old) <= 1e-6 * new
    h = h[:-1]
    assert abs(h[-10:].mean() - h[-20:-10].mean()) > 1e-6 * h[-10:].mean()   # not one check earlier
