"""Steady-flux driver for batched sweeps.

Advances an ``lbm.Batch`` in blocks of ``check_every`` steps, records the flux
Q of eq. (11) of every channel after each block, and retires a channel once
its flux has stopped changing: |Q(t) - Q(t - window)| <= rtol * |Q(t)|.
With ``average`` (for 16-bit storage with stochastic rounding, whose flux keeps
a small rounding noise) the mean of the records of the last window is compared
with the mean of the window before, and that mean is the reported flux.
All stepping and reductions run on the GPU; this module only decides when to
stop and keeps the history.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class SweepResult:
    steps: np.ndarray              # steps taken by each channel when it was retired
    Q: np.ndarray                  # flux at retirement (the converged value)
    converged: np.ndarray          # bool: met the criterion before max_steps
    history: list = field(default_factory=list)   # per channel: list of (step, Q)
    node_updates: float = 0.0      # sum over channels of nodes * steps

    def steps_to_within(self, i: int, Q_ref: float, rtol: float) -> int:
        """First recorded step after which every later record of channel i is
        within rtol of Q_ref; -1 if never."""
        hist = self.history[i]
        ok = [abs(q - Q_ref) <= rtol * abs(Q_ref) for _, q in hist]
        t = -1
        for k in range(len(hist) - 1, -1, -1):
            if not ok[k]:
                break
            t = hist[k][0]
        return t


def run_to_steady(batch, check_every: int = 100, window: int = 1000, rtol: float = 1e-8,
                  max_steps: int = 200_000, graph_steps: int | None = None,
                  min_steps: int = 0, log=None, log_every: int = 5000, average: bool = False) -> SweepResult:
    """Step every channel of ``batch`` until its flux is steady (see module doc);
    ``log`` (if given) receives a progress line every ``log_every`` steps."""
    n = batch.n
    if graph_steps is None:
        graph_steps = check_every if check_every % 2 == 0 else 0
    batch.set_graph(graph_steps)
    lag = max(1, window // check_every)
    hist = [[] for _ in range(n)]
    active = np.ones(n, bool)
    steps = np.zeros(n, np.int64)
    Qfin = np.full(n, np.nan)
    conv = np.zeros(n, bool)
    nodes = np.array([ny * nx for ny, nx in batch.shapes], np.float64)
    t = 0
    while active.any() and t < max_steps:
        batch.step(check_every)
        t += check_every
        Q, _, status = batch.flux_nocheck()
        done = np.zeros(n, bool)
        for i in np.nonzero(active)[0]:
            hist[i].append((t, float(Q[i])))
            if not np.isfinite(Q[i]):
                done[i] = True          # diverged: stop it, not converged
                continue
            if t < min_steps:
                continue
            if average:
                if len(hist[i]) >= 2 * lag:
                    new = float(np.mean([q for _, q in hist[i][-lag:]]))
                    old = float(np.mean([q for _, q in hist[i][-2 * lag:-lag]]))
                    if abs(new - old) <= rtol * abs(new):
                        done[i] = True
                        conv[i] = True
            elif len(hist[i]) > lag:
                q_old = hist[i][-1 - lag][1]
                if abs(Q[i] - q_old) <= rtol * abs(Q[i]):
                    done[i] = True
                    conv[i] = True
        for i in np.nonzero(done)[0]:
            steps[i] = t
            last = [q for _, q in hist[i][-lag:]]
            Qfin[i] = float(np.mean(last)) if average and conv[i] else hist[i][-1][1]
        if done.any():
            active &= ~done
            batch.retire(~active)
        if log and t % log_every == 0:
            log(f"  step {t}: {int(active.sum())} of {n} channels still running")
    for i in np.nonzero(active)[0]:
        steps[i] = t
        Qfin[i] = hist[i][-1][1] if hist[i] else np.nan
    return SweepResult(steps=steps, Q=Qfin, converged=conv, history=hist,
                       node_updates=float((nodes * steps).sum()))
