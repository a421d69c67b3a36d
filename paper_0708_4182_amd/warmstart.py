"""Learned warm start of steady channel flow.

A convolutional encoder-decoder (include/lbm_net.h) maps a channel's wall mask,
electric force f and interaction strength G to its steady density and velocity;
the lattice is then initialised at the equilibrium of that prediction and the
plain lattice Boltzmann steps decide the result.  The quantity of interest is
the number of lattice updates until the flux of eq. (11) is steady:

  - Q_inf is the flux of the cold (standard) start run until it changes by at
    most 1e-8 relative over 1000 steps;
  - a run is steady at the first check (every 100 steps) from which every check
    of the next 5000 steps lies within 1e-4 of Q_inf.

Every warm-started run is measured against the cold start's Q_inf, so a poor
prediction costs steps, never accuracy; a run that does not settle on Q_inf
(another steady branch) is counted as a failure.  The lattice conserves mass,
so the seeded density is scaled to the cold start's mass (otherwise the warm
run would settle on the steady state of another mass); a prediction that is
not finite is discarded and the channel starts cold.

Data movement (batching, normalisation) uses torch; the network's forward and
backward passes and the Adam updates run in the library's HIP kernels, and
every lattice step in its lattice kernels.
"""
from __future__ import annotations

import json
import math
import time
from dataclasses import dataclass

import numpy as np

from . import inputs as I
from . import lbm, net, sweep

F_SCALE = 3e-3          # f of the data set lies in [0, 3e-3)
G_MID, G_HALF = -5.0, 0.5
STEADY_RTOL, STEADY_HOLD = 1e-4, 5000


# ------------------------------------------------------------------- steadiness
def steady_time(hist, Q_ref: float, rtol: float = STEADY_RTOL, hold: int = STEADY_HOLD) -> int:
    """First recorded step t from which every record in [t, t + hold] is within
    rtol of Q_ref, the history reaching t + hold; -1 if there is none."""
    t = np.array([h[0] for h in hist], np.int64)
    q = np.array([h[1] for h in hist], np.float64)
    if len(t) == 0 or not np.isfinite(Q_ref):
        return -1
    ok = np.abs(q - Q_ref) <= rtol * abs(Q_ref)
    start = None
    for k in range(len(t)):
        if not ok[k]:
            start = None
            continue
        if start is None:
            start = t[k]
        if t[k] - start >= hold:
            return int(start)
    return -1


def run_until_steady(batch, Q_ref, rtol: float = STEADY_RTOL, hold: int = STEADY_HOLD,
                     check_every: int = 100, max_steps: int = 100_000, graph_steps: int | None = None,
                     log=None, log_every: int = 5000):
    """Step every channel until it meets the steadiness rule against Q_ref[i]
    (then it is retired) or max_steps; returns (steady step or -1, histories)."""
    n = batch.n
    Q_ref = np.asarray(Q_ref, np.float64)
    batch.set_graph(check_every if graph_steps is None else graph_steps)
    hist = [[] for _ in range(n)]
    since = [None] * n
    result = np.full(n, -1, np.int64)
    active = np.ones(n, bool)
    t = 0
    while active.any() and t < max_steps:
        batch.step(check_every)
        t += check_every
        Q, _, _ = batch.flux_nocheck()
        done = np.zeros(n, bool)
        for i in np.nonzero(active)[0]:
            hist[i].append((t, float(Q[i])))
            if not np.isfinite(Q[i]):
                done[i] = True
                continue
            if abs(Q[i] - Q_ref[i]) <= rtol * abs(Q_ref[i]):
                if since[i] is None:
                    since[i] = t
                if t - since[i] >= hold:
                    result[i] = since[i]
                    done[i] = True
            else:
                since[i] = None
        if done.any():
            active &= ~done
            batch.retire(~active)
        if log and t % log_every == 0:
            log(f"  step {t}: {int(active.sum())} of {n} channels not yet steady")
    return result, hist


# --------------------------------------------------------------------- features
def features(cases):
    """Network inputs [n][3][ny][nx] float32 (solid mask, f / 3e-3, (G + 5) / 0.5)
    and fluid masks [n][ny][nx] uint8."""
    n = len(cases)
    ny, nx = cases[0].solid.shape
    X = np.empty((n, 3, ny, nx), np.float32)
    fluid = np.empty((n, ny, nx), np.uint8)
    for i, c in enumerate(cases):
        X[i, 0] = c.solid
        X[i, 1] = c.params.f_elec / F_SCALE
        X[i, 2] = (c.meta["G"] - G_MID) / G_HALF
        fluid[i] = c.solid == 0
    return X, fluid


@dataclass
class Scales:
    """Per-plane affine normalisation of the targets (rho, ux, uy)."""
    mean: np.ndarray
    std: np.ndarray

    @staticmethod
    def fit(T, fluid):
        m = fluid.astype(bool)
        mean = np.array([T[:, p][m].mean(dtype=np.float64) for p in range(3)])
        std = np.array([T[:, p][m].std(dtype=np.float64) for p in range(3)])
        return Scales(mean, np.maximum(std, 1e-30))

    def to_dict(self):
        return {"mean": self.mean.tolist(), "std": self.std.tolist()}

    @staticmethod
    def from_dict(d):
        return Scales(np.array(d["mean"]), np.array(d["std"]))


# ------------------------------------------------------------------ steady data
def steady_states(cases, check_every: int = 100, window: int = 1000, rtol: float = 1e-8,
                  max_steps: int = 100_000, log=None):
    """Cold-start every case to a steady flux (FP32 storage) in one batch.

    Returns a dict: T [n][3][ny][nx] float32 steady (rho, ux, uy); Q (Q_inf);
    converged; cold (steady step per the rule of this module, -1 if none);
    steps (steps run)."""
    t0 = time.perf_counter()
    b = lbm.Batch(cases)
    res = sweep.run_to_steady(b, check_every=check_every, window=window, rtol=rtol, max_steps=max_steps,
                              log=log)
    ny, nx = cases[0].solid.shape
    T = np.empty((len(cases), 3, ny, nx), np.float32)
    for i in range(len(cases)):
        T[i] = b.moments_device(i).cpu().numpy()
    cold = np.array([steady_time(res.history[i], res.Q[i]) for i in range(len(cases))], np.int64)
    del b
    if log:
        log(f"steady states: {len(cases)} channels, {int(res.steps.max())} steps max, "
            f"{int(res.converged.sum())} converged, {time.perf_counter() - t0:.1f} s")
    return dict(T=T, Q=res.Q, converged=res.converged, cold=cold, steps=res.steps)


# ---------------------------------------------------------------------- training
def train(model, X, T, fluid, epochs: int, batch: int, lr: float = 1e-3, lr_min: float = 1e-5,
          seed: int = 0, log=None, log_every: int = 50):
    """Adam on minibatches of (X, T, fluid) device tensors (T normalised), cosine
    learning-rate decay from lr to lr_min; returns the logged losses."""
    import torch
    n = X.shape[0]
    per_epoch = n // batch
    total = epochs * per_epoch
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    losses = []
    it = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=gen, device=X.device)
        for k in range(per_epoch):
            idx = perm[k * batch:(k + 1) * batch]
            xb = X.index_select(0, idx).contiguous()
            tb = T.index_select(0, idx).contiguous()
            fb = fluid.index_select(0, idx).contiguous()
            a = lr_min + 0.5 * (lr - lr_min) * (1 + math.cos(math.pi * it / max(1, total)))
            want = it % log_every == 0 or it == total - 1
            loss = model.train_step(xb, tb, fb, lr=a, want_loss=want)
            if want:
                losses.append((it, loss))
                if log:
                    log(f"  it {it:6d}/{total} epoch {ep} lr {a:.2e} loss {loss:.4e} "
                        f"({time.perf_counter() - t0:.1f} s)")
            it += 1
    torch.cuda.synchronize()
    return losses


def predict(model, X, scales: Scales):
    """Physical (rho, ux, uy) [n][3][ny][nx] predicted for device inputs X."""
    import torch
    out = torch.empty((X.shape[0], 3) + tuple(X.shape[2:]), dtype=torch.float32, device=X.device)
    for k in range(0, X.shape[0], model.batch):
        out[k:k + model.batch] = model.forward(X[k:k + model.batch].contiguous())
    mean = torch.tensor(scales.mean, dtype=torch.float32, device=X.device).view(1, 3, 1, 1)
    std = torch.tensor(scales.std, dtype=torch.float32, device=X.device).view(1, 3, 1, 1)
    return out * std + mean


def normalised_mse(pred, T, fluid, scales: Scales):
    """Mean over fluid nodes of ((pred - T) / std)^2, per plane (rho, ux, uy)."""
    m = fluid.to(pred.dtype)
    return [float((((pred[:, p] - T[:, p]) / float(scales.std[p])) ** 2 * m).sum() / m.sum())
            for p in range(3)]


U_MAX = 0.1             # lattice speed cap for a seeded velocity (Mach ~ 0.17)


def warm_fields(pred: np.ndarray, solid: np.ndarray, G: float, mass: float, mode: str = "flow",
                rho_cold: np.ndarray | None = None):
    """Initial (rho, ux, uy) [3][ny][nx] float32 from a prediction, or None if
    the prediction is not finite on the fluid.

    The lattice conserves mass exactly, so the steady state reached depends on
    the initial mass, which must be the cold start's fluid mass ``mass``:
      - mode "raw": the predicted density, clipped to [rho_v / 2, 1.5 rho_l] of
        the coexistence pair at G, scaled to ``mass``;
      - mode "snap": each fluid node takes the phase of its predicted density
        (vapour below the mean of rho_v and rho_l, liquid otherwise) at the
        coexistence density rho_v, and the liquid density is set so that the
        mass is ``mass``: a sharp phase map like the cold start's;
      - mode "flow": the cold start's own density ``rho_cold`` (so its phase
        map and mass), with the predicted velocity.
    The velocity is clipped to |u_x|, |u_y| <= U_MAX; solid nodes get 0."""
    fl = solid == 0
    if not all(np.isfinite(pred[p][fl]).all() for p in range(3)):
        return None
    rv, rl = I.coexistence(G)
    if mode == "raw":
        rho = np.where(fl, np.clip(pred[0].astype(np.float64), 0.5 * rv, 1.5 * rl), 0.0)
        rho *= mass / rho[fl].sum()
    elif mode == "snap":
        liquid = fl & (pred[0] >= 0.5 * (rv + rl))
        vapour = fl & ~liquid
        n_l = int(liquid.sum())
        rho_l = (mass - rv * vapour.sum()) / n_l if n_l else rl
        if not rho_l > 0:
            return None
        rho = np.where(liquid, rho_l, np.where(vapour, rv, 0.0))
    elif mode == "flow":
        rho = np.where(fl, rho_cold, 0.0)
    else:
        raise ValueError(f"unknown mode {mode!r}")
    ux = np.where(fl, np.clip(pred[1], -U_MAX, U_MAX), 0.0)
    uy = np.where(fl, np.clip(pred[2], -U_MAX, U_MAX), 0.0)
    return np.stack([rho, ux, uy]).astype(np.float32)


# -------------------------------------------------------------------- evaluation
def warm_vs_cold(model, scales: Scales, cases, Q_inf, cold, max_steps: int = 100_000, log=None,
                 pred=None, mode: str = "flow"):
    """Warm-start every case from the network and time it to steadiness against
    the cold start's Q_inf; ``cold`` holds the cold start's steady steps."""
    import torch
    X, fluid = features(cases)
    Xd = torch.from_numpy(X).cuda()
    if pred is None:
        pred = predict(model, Xd, scales)
    P = pred.cpu().numpy()
    b = lbm.Batch(cases)
    used = np.zeros(len(cases), bool)
    seeded = []
    for i, c in enumerate(cases):
        mass = float(c.rho[c.solid == 0].sum())
        F = warm_fields(P[i], c.solid, c.meta["G"], mass, mode, rho_cold=c.rho)
        if F is not None:
            Fd = torch.from_numpy(F).to(pred.device)
            seeded.append(Fd)
            b.init_device(i, Fd[0], Fd[1], Fd[2])
            used[i] = True
    Q0, _, _ = b.flux_nocheck()           # flux of the initial (seeded) state; synchronizes
    del seeded
    warm, hist = run_until_steady(b, Q_inf, max_steps=max_steps, log=log)
    del b
    Q_inf = np.asarray(Q_inf)
    Q_end = np.array([h[-1][1] if h else np.nan for h in hist])
    surrogate = np.abs(Q0 - Q_inf) / np.abs(Q_inf)
    ok = (warm >= 0) & (cold >= 0)
    fail_w = int(((warm < 0) & (cold >= 0)).sum())
    fail_c = int((cold < 0).sum())
    nodes = float(cases[0].solid.size)
    stats = dict(
        mode=mode, n=len(cases), used_prediction=int(used.sum()),
        warm_failures=fail_w, cold_failures=fail_c,
        median_cold_steps=float(np.median(cold[ok])) if ok.any() else None,
        median_warm_steps=float(np.median(warm[ok])) if ok.any() else None,
        median_speedup=float(np.median(cold[ok] / np.maximum(warm[ok], 100))) if ok.any() else None,
        total_cold_updates=float(cold[ok].sum() * nodes),
        total_warm_updates=float(warm[ok].sum() * nodes),
        surrogate_flux_error_median=float(np.median(surrogate[used])) if used.any() else None,
        surrogate_flux_error_p90=float(np.percentile(surrogate[used], 90)) if used.any() else None,
        failed_end_offset_median=(float(np.median(np.abs(Q_end[warm < 0] / Q_inf[warm < 0] - 1)))
                                  if (warm < 0).any() else None),
    )
    if log:
        log("warm vs cold: " + json.dumps(stats))
    return stats, warm, surrogate, Q_end


# ----------------------------------------------------------- branch detection
def phase_mismatch(rho, rho_pred, solid, G: float) -> int:
    """Fluid nodes whose phase (liquid: rho >= (rho_v + rho_l) / 2 at G) in
    ``rho`` differs from the phase in the prediction ``rho_pred``, not counting
    nodes next to an interface of the prediction (within one node of a node of
    the other phase), where the phase of a diffuse interface is ambiguous."""
    rv, rl = I.coexistence(G)
    mid = 0.5 * (rv + rl)
    fl = solid == 0
    liq_p = (rho_pred >= mid) & fl
    liq = (rho >= mid) & fl
    # nodes of the prediction with a neighbour (8-connected, periodic in x) of the other phase
    edge = np.zeros_like(fl)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            nb = np.roll(np.roll(liq_p, dx, axis=1), dy, axis=0)
            nfl = np.roll(np.roll(fl, dx, axis=1), dy, axis=0)
            edge |= nfl & (nb != liq_p)
    return int(((liq != liq_p) & fl & ~edge).sum())


def warm_with_fallback(model, scales: Scales, cases, check_every: int = 100, window: int = 1000,
                       rtol: float = 1e-8, max_steps: int = 100_000, q_margin: float = 0.02,
                       phase_margin: int = 8, mode: str = "flow", pred=None, t_cold: int = 0, log=None):
    """Warm-start every case from the network and run it to a steady flux by
    its own rule (|Q(t) - Q(t - window)| <= rtol |Q|, as the cold runs), without
    any cold reference.

    With t_cold > 0 every channel first runs t_cold steps from its cold start,
    and the prediction's velocity is then seeded onto the density it has
    reached (mode "flow"): the early cold transient is where a channel's
    steady branch (how its cavities and films form) is decided, and the
    prediction then only shortens the slow viscous decay that follows.

    A settled warm channel is accepted when its flux is within q_margin of the
    flux of the seeded state and at most phase_margin fluid nodes away from the
    predicted interfaces have the other phase; otherwise it is flagged as
    settled on another steady branch, re-initialised cold (the case's initial
    fields) inside the same batch, and run to its own steady flux.  A
    prediction that is not finite starts cold.

    Returns per-channel arrays: steps (lattice steps run: the cold prefix,
    warm, and any cold restart), Q (accepted flux), flagged, Q_warm (settled
    warm flux, NaN if none), Q_pred (flux of the seeded state), mismatch
    (phase mismatch at settling)."""
    import torch
    n = len(cases)
    X, fluid = features(cases)
    Xd = torch.from_numpy(X).cuda()
    if pred is None:
        pred = predict(model, Xd, scales)
    P = pred.cpu().numpy()
    b = lbm.Batch(cases)
    rho_start = [c.rho for c in cases]
    if t_cold > 0:
        b.set_graph(100 if t_cold % 100 == 0 else 0)
        b.step(t_cold)
        rho_start = [b.moments_device(i)[0].cpu().numpy().astype(np.float64) for i in range(n)]
    seeded = []
    warm = np.zeros(n, bool)
    for i, c in enumerate(cases):
        mass = float(c.rho[c.solid == 0].sum())
        F = warm_fields(P[i], c.solid, c.meta["G"], mass, mode, rho_cold=rho_start[i])
        if F is not None:
            Fd = torch.from_numpy(F).to(pred.device)
            seeded.append(Fd)
            b.init_device(i, Fd[0], Fd[1], Fd[2])
            warm[i] = True
    Q_pred, _, _ = b.flux_nocheck()           # synchronizes; the seeded states are read
    del seeded
    b.set_graph(check_every if check_every % 2 == 0 else 0)
    lag = max(1, window // check_every)
    hist = [[] for _ in range(n)]
    active = np.ones(n, bool)
    steps = np.full(n, int(t_cold), np.int64)
    flagged = np.zeros(n, bool)
    Q_out = np.full(n, np.nan)
    Q_warm = np.full(n, np.nan)
    mism = np.full(n, -1, np.int64)
    cold_fields = {}
    t = 0
    while active.any() and t < max_steps:
        b.step(check_every)
        t += check_every
        steps[active] += check_every
        Q, _, _ = b.flux_nocheck()
        settled = []
        for i in np.nonzero(active)[0]:
            hist[i].append(float(Q[i]))
            if not np.isfinite(Q[i]):
                settled.append(i)
                continue
            if len(hist[i]) > lag and abs(Q[i] - hist[i][-1 - lag]) <= rtol * abs(Q[i]):
                settled.append(i)
        retire = np.zeros(n, bool)
        for i in settled:
            if warm[i] and not flagged[i]:
                Q_warm[i] = Q[i]
                rho = b.moments_device(i)[0].cpu().numpy()
                mism[i] = phase_mismatch(rho, P[i][0], cases[i].solid, cases[i].meta["G"])
                off = abs(Q[i] - Q_pred[i]) > q_margin * abs(Q_pred[i])
                if off or mism[i] > phase_margin or not np.isfinite(Q[i]):
                    flagged[i] = True
                    c = cases[i]
                    fields = torch.from_numpy(np.stack([c.rho, c.ux, c.uy]).astype(np.float32)).cuda()
                    cold_fields[i] = fields
                    b.init_device(i, fields[0], fields[1], fields[2])
                    hist[i] = []
                    continue
            Q_out[i] = Q[i]
            retire[i] = True
        if retire.any():
            active &= ~retire
            b.retire(~active)
        if log and t % 5000 == 0:
            log(f"  step {t}: {int(active.sum())} of {n} channels running, {int(flagged.sum())} restarted cold")
    for i in np.nonzero(active)[0]:
        Q_out[i] = hist[i][-1] if hist[i] else np.nan
    del b, cold_fields
    return dict(steps=steps, Q=Q_out, flagged=flagged, Q_warm=Q_warm, Q_pred=np.asarray(Q_pred),
                mismatch=mism, warm=warm, converged=~active)
