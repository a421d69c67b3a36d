"""Experiments of the paper run on the GPU library (no oracle involved).

  flux_vs_field   Q/Q0 against the electric force f in a rough-wall channel
                  (the paper's Fig. 8 experiment; every f is one channel of a
                  batch, all advanced together to steady flux).
  sweep_throughput aggregate MLUPS of the batched engine on the 256-channel
                  sweep table (uneven widths, lengths, roughness, f and G).
  sweep_steady    the sweep table driven to steady flux: steps, lattice
                  updates and wall time per channel.
  warm_start      train the encoder-decoder on steady channels and compare
                  lattice updates to steady flux, warm start against cold.
  channel_study   rough channels of the paper's widths 80 and 160 over a
                  sweep of f, to steady flux: Q/Q0 and velocity profiles.
  small_configs   the launch-bound 128x64 and 1024x128 lattices, ordinary
                  launches against hipGraph replays.
  net_throughput  training and inference rate of the warm-start network.

Run as ``python -m paper_0708_4182_amd.experiments <name> [key=value ...]``;
prints JSON.
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

from . import inputs as I
from . import lbm
from .sweep import run_to_steady


def flux_vs_field(nx=1024, ny=128, fs=(0.0, 5e-4, 1e-3, 1.5e-3, 2e-3), seed=0, storage=0,
                  max_steps=100_000, rtol=1e-8, accel=1e-6):
    cases = [I.rough_channel_case(nx=nx, ny=ny, f_elec=f, seed=seed, accel=accel, storage=storage)
             for f in fs]
    b = lbm.Batch(cases)
    t0 = time.perf_counter()
    res = run_to_steady(b, check_every=200, window=2000, rtol=rtol, max_steps=max_steps)
    dt = time.perf_counter() - t0
    Q = res.Q
    return {"experiment": "flux_vs_field", "nx": nx, "ny": ny, "seed": seed, "storage": storage,
            "f": list(fs), "Q": Q.tolist(), "Q_over_Q0": (Q / Q[0]).tolist(),
            "steps": res.steps.tolist(), "converged": res.converged.tolist(), "seconds": dt}


def sweep_throughput(n=256, seed=0, storage=1, steps=60, warmup=20, graph=10, tune=True, rounding=1, tile="",
                     kernel=""):
    """The sweep table's batched step: time per step over ``steps`` steps (hipGraph
    replays of ``graph`` steps).  ``tile`` "block_x,rows" fixes the tile (no
    autotune trial launches, for profiler traces); else ``tune`` autotunes
    (steps per launch included).  ``kernel`` ("fused", "two", "three") then
    fixes the steps per launch."""
    import torch
    rows = I.sweep_table(n, seed)
    cases = [I.sweep_case(r, storage=storage, rounding=rounding) for r in rows]
    nodes = sum(c.params.nx * c.params.ny for c in cases)
    fluid = sum(int((c.solid == 0).sum()) for c in cases)
    b = lbm.Batch(cases)
    if tile:
        bx, r = (int(v) for v in str(tile).split(","))
        b.set_tile(bx, r)
        tile = [bx, r]
    elif tune:
        bx, r, us = b.autotune(reps=3)
        tile = [bx, r]
    else:
        tile = None
    if kernel:
        b.set_kernel(kernel)
    b.set_graph(graph)
    b.step(warmup)
    b.flux()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(b.stream)
    b.step(steps)
    e1.record(b.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    es = {0: 4, 1: 2, 2: 2}[storage]
    return {"experiment": "sweep_throughput", "channels": n, "nodes": nodes, "fluid_nodes": fluid,
            "storage": storage, "rounding": rounding, "tile": tile, "kernel": b.kernel(), "graph_steps": graph,
            "ms_per_step": ms,
            "mlups": nodes / (ms * 1e-3) / 1e6,
            "achieved_GBs": 18 * es * fluid / (ms * 1e-3) / 1e9}


def small_configs(steps=2000, warmup=200, graph=50):
    """Launch-bound workloads: the 128 x 64 droplet (config 1) and the
    1024 x 128 rough channel (config 2), FP32, each timed with ordinary
    lbm_step launches and with hipGraph replays of ``graph`` steps
    (lbm_set_graph).  MLUPS over all nodes."""
    import torch
    out = {}
    for name, case in (("droplet128x64", I.droplet_case(f_elec=1e-3)),
                       ("rough1024x128", I.rough_channel_case(nx=1024, ny=128, f_elec=1e-3, seed=0))):
        nodes = case.params.nx * case.params.ny
        res = {}
        for mode in ("eager", "graph"):
            sim = lbm.from_case(case)
            sim.autotune(reps=20)
            if mode == "graph":
                sim.set_graph(graph)
            run, stream = sim.step, sim.stream
            run(warmup)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run(steps)
            e1.record(stream)
            torch.cuda.synchronize()
            us = 1000.0 * e0.elapsed_time(e1) / steps
            res[mode] = {"us_per_step": round(us, 2), "mlups": round(nodes / us, 1)}
            del sim
        out[name] = res
    return out


def channel_study(widths="80,160", forces="", nx=256, storage=0, max_steps=400_000, check_every=200,
                  window=4000, rtol=1e-8, layers=2, out="", reading="configs"):
    """Rough channels of the paper's two widths (steps a = 8, b = 4, p = 32 on
    both walls, both walls electrodes) over a sweep of the electric force, all
    in one batch driven to steady flux: Q / Q0 per width and the
    channel-averaged velocity profiles (the paper's flux and velocity figures).
    reading "configs": the normalisation of reading R1 (G = -5), fields
    0..3e-3 on ``layers`` layers; reading "paper": the paper's own parameters
    under reading R29 (calG = -0.52, w = -0.14, tau = 0.9, f_b = 8e-6), its
    fields 0..0.25 on the single layer next to the walls.  Writes
    profiles.npz and study.json under ``out`` if given."""
    import json
    import os
    import torch
    if not forces:
        forces = "0,0.05,0.1,0.15,0.2,0.25" if reading == "paper" else "0,5e-4,1e-3,1.5e-3,2e-3,3e-3"
    ws = [int(v) for v in str(widths).split(",")]
    fs = [float(v) for v in str(forces).split(",")]
    cases, keys = [], []
    for w in ws:
        for f in fs:
            if reading == "paper":
                cases.append(I.paper_channel_case(nx=nx, ny=w, f_elec=f, seed=0, storage=storage))
            else:
                cases.append(I.rough_channel_case(nx=nx, ny=w, f_elec=f, seed=0, layers=layers, storage=storage))
            keys.append((w, f))
    b = lbm.Batch(cases)
    b.autotune(reps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run_to_steady(b, check_every=check_every, window=window, rtol=rtol, max_steps=max_steps,
                        log=lambda m: print("#", m, flush=True), log_every=20_000)
    wall = time.perf_counter() - t0
    prof = [b.profile(i) for i in range(len(cases))]
    table = {}
    for w in ws:
        q0 = res.Q[keys.index((w, 0.0))] if 0.0 in fs else float("nan")
        table[w] = {f"{f:g}": {"Q": float(res.Q[keys.index((w, f))]),
                               "Q_over_Q0": float(res.Q[keys.index((w, f))] / q0),
                               "steps": int(res.steps[keys.index((w, f))]),
                               "converged": bool(res.converged[keys.index((w, f))])} for f in fs}
    asym = {}
    for i, (w, f) in enumerate(keys):
        # liquid nodes in the lower half minus the upper half, over all liquid nodes: 0 for a
        # liquid that stays in the middle, +-1 for one absorbed by one wall
        rho = b.moments(i)[0]
        fluid = cases[i].solid == 0
        liq = (rho >= cases[i].params.rho_c) & fluid
        lo, hi = liq[: w // 2].sum(), liq[w // 2:].sum()
        asym[f"{w}/{f:g}"] = float((lo - hi) / max(lo + hi, 1))
    summary = {"experiment": "channel_study", "reading": reading, "nx": nx, "widths": ws, "forces": fs,
               "storage": storage, "layers": 1 if reading == "paper" else layers, "wall_s": wall,
               "node_updates": res.node_updates, "table": table, "liquid_asymmetry": asym}
    if out:
        os.makedirs(out, exist_ok=True)
        np.savez(os.path.join(out, "profiles.npz"), keys=np.array(keys), **{f"p{i}": p for i, p in enumerate(prof)})
        with open(os.path.join(out, "study.json"), "w") as fh:
            json.dump(summary, fh, indent=1)
    return summary


def net_flops(H=64, W=256, cin=3, cout=3, chans=(32, 64, 128, 128)):
    """(forward, backward) multiply-add FLOPs of one sample of the warm-start
    network: 2 k^2 cin cout per output pixel and layer; the backward does the
    input gradient (all layers but the first) and the weight gradient."""
    from . import net
    sizes = [(H, W)] * 2 + [(H // 2, W // 2)] * 2 + [(H // 4, W // 4)] * 2 + [(H // 8, W // 8)] * 2 \
        + [(H // 4, W // 4)] * 2 + [(H // 2, W // 2)] * 2 + [(H, W)] * 3
    fwd = bwd = 0.0
    for i, ((_, ci, co, k), (h, w)) in enumerate(zip(net.layer_shapes(cin, cout, chans), sizes)):
        f = 2.0 * k * k * ci * co * h * w
        fwd += f
        bwd += f * (2 if i > 0 else 1)
    return fwd, bwd


def net_throughput(batch=32, H=64, W=256, steps=50, warmup=5, seed=0):
    """Training steps (forward, backward, Adam) and inference of the warm-start
    network on random inputs of the warm-start shape, bf16 activations:
    samples per second and delivered TFLOP/s."""
    import torch
    from . import net
    m = net.Net(H, W, batch, act_bf16=True)
    m.set_params(net.he_init(net.layer_shapes(), seed))
    g = torch.Generator(device="cuda").manual_seed(seed)
    x = torch.randn((batch, 3, H, W), generator=g, device="cuda")
    t = torch.randn((batch, 3, H, W), generator=g, device="cuda")
    fluid = (torch.rand((batch, H, W), generator=g, device="cuda") > 0.1).to(torch.uint8)
    fwd, bwd = net_flops(H, W)
    out = {}
    for mode in ("train", "infer"):
        run = (lambda: m.train_step(x, t, fluid, lr=1e-4, want_loss=False)) if mode == "train" \
            else (lambda: m.forward(x))
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(m.stream)
        for _ in range(steps):
            run()
        e1.record(m.stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        flops = batch * (fwd + bwd if mode == "train" else fwd)
        out[mode] = {"ms_per_batch": round(ms, 3), "samples_per_s": round(batch / (ms * 1e-3), 1),
                     "tflops": round(flops / (ms * 1e-3) / 1e12, 2)}
    out["gflop_per_sample"] = {"forward": round(fwd / 1e9, 3), "backward": round(bwd / 1e9, 3)}
    return out


def sweep_steady(n=256, seed=0, storage=1, max_steps=200_000, check_every=200, window=2000, rtol=None,
                 rounding=1):
    """The 256-channel sweep table driven to steady flux in one batch (kernel,
    with one, two or three steps per launch, schedule and tile autotuned;
    hipGraph of check_every steps, channels retired as they converge):
    per-channel steps, lattice updates and wall time.  16-bit
    channels use stochastic rounding by default: with nearest rounding a
    16-bit lattice settles on an exact fixed point that carries the rounding
    bias (on the first 32 channels of the table, fluxes 18% off the FP32 ones
    at the median after 100,000 steps, against 2.5e-4 with stochastic
    rounding).  Stochastic rounding leaves a small noise in the flux, so the
    averaged steady rule applies (window means, rtol 1e-5); nearest rounding
    and FP32 keep the plain rule at rtol 1e-8."""
    import torch
    rows = I.sweep_table(n, seed)
    cases = [I.sweep_case(r, storage=storage, rounding=rounding) for r in rows]
    b = lbm.Batch(cases)
    bx, r, us = b.autotune(reps=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    average = storage != 0 and rounding == 1
    if rtol is None:
        rtol = 1e-5 if average else 1e-8
    res = run_to_steady(b, check_every=check_every, window=window, rtol=rtol, max_steps=max_steps,
                        log=lambda m: print("#", m, flush=True), log_every=20_000, average=average)
    wall = time.perf_counter() - t0
    from .warmstart import steady_time
    nodes = np.array([c.params.nx * c.params.ny for c in cases], np.float64)
    widths = np.array([c.params.ny for c in cases])
    conv = res.converged
    # the steady time of the warm-start comparison: within 1e-4 of the final flux for 5000 steps
    st = np.array([steady_time(res.history[i], res.Q[i]) for i in range(n)])
    return {"experiment": "sweep_steady", "channels": n, "storage": storage, "rounding": rounding,
            "steady_rule": {"rtol": rtol, "averaged": average}, "kernel": b.kernel(), "tile": [bx, r],
            "max_steps": max_steps, "converged": int(conv.sum()),
            "steps_median": float(np.median(res.steps)), "steps_max": int(res.steps.max()),
            "lattice_updates": res.node_updates, "wall_seconds": wall,
            "steady_1e-4_found": int((st >= 0).sum()),
            "steady_1e-4_median_steps": float(np.median(st[st >= 0])) if (st >= 0).any() else None,
            "lattice_updates_to_steady_1e-4": float((nodes * np.where(st >= 0, st, res.steps)).sum()),
            "mlups_during_sweep": res.node_updates / wall / 1e6,
            "unconverged_widths": sorted(int(w) for w in widths[~conv]),
            "converged_width_max": int(widths[conv].max()) if conv.any() else None,
            "per_channel": [{"ny": int(c.params.ny), "nx": int(c.params.nx), "steps": int(sp),
                             "converged": bool(cv), "steady_1e-4": int(t4), "Q": float(q)}
                            for c, sp, cv, t4, q in zip(cases, res.steps, conv, st, res.Q)]}


def warm_start(train=4096, test=512, nx=256, ny=64, epochs=30, batch=32, lr=1e-3, lr_min=1e-5,
               bf16=1, chans="32,64,128,128", max_steps=100_000, seed=0, out="", modes="flow,snap,raw",
               params=""):
    """Learned warm start: steady states of train + test channels (cold starts),
    training of the encoder-decoder on the first ``train`` seeds, and the
    warm-vs-cold comparison on the next ``test`` seeds."""
    import os

    import torch

    from . import net, warmstart as WS

    def log(msg):
        print(f"# {msg}", flush=True)

    chans = tuple(int(c) for c in str(chans).split(","))
    seeds = list(range(train + test))
    cases = [I.warm_case(s, nx=nx, ny=ny) for s in seeds]
    log(f"{len(cases)} channels {nx}x{ny}: steady states (cold starts)")
    data = WS.steady_states(cases, max_steps=max_steps, log=log)
    X, fluid = WS.features(cases)
    T = data["T"]
    scales = WS.Scales.fit(T[:train], fluid[:train])
    Tn = (T - scales.mean.reshape(1, 3, 1, 1)) / scales.std.reshape(1, 3, 1, 1)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(Tn.astype(np.float32)).cuda()
    Fd = torch.from_numpy(fluid).cuda()
    model = net.Net(ny, nx, batch, chans=chans, act_bf16=bool(int(bf16)))
    if params:
        theta = np.load(params) if params.endswith(".npy") else np.fromfile(params, np.float32)
        model.set_params(theta)
        log(f"parameters loaded from {params}; no training")
        losses, train_s, epochs = [(0, float("nan"))], float("nan"), 0
    else:
        model.set_params(net.he_init(net.layer_shapes(chans=chans), seed))
        log(f"training: {model.n_params} parameters, {epochs} epochs of {train // batch} steps")
        t0 = time.perf_counter()
        losses = WS.train(model, Xd[:train], Td[:train], Fd[:train], epochs, batch, lr, lr_min, seed,
                          log=log)
        train_s = time.perf_counter() - t0
    pred = WS.predict(model, Xd[train:], scales)
    Ttest = torch.from_numpy(T[train:]).cuda()
    test_mse = WS.normalised_mse(pred, Ttest, Fd[train:], scales)
    log(f"test MSE per normalised plane {test_mse}")
    res = {"experiment": "warm_start", "nx": nx, "ny": ny, "train": train, "test": test,
           "epochs": epochs, "batch": batch, "bf16_activations": bool(int(bf16)), "chans": chans,
           "params": model.n_params, "train_seconds": train_s,
           "train_steps_per_s": epochs * (train // batch) / train_s if epochs else None,
           "final_train_loss": losses[-1][1], "test_mse_normalised": test_mse,
           "cold_converged": int(data["converged"].sum()), "scales": scales.to_dict(), "results": []}
    per_seed = dict(seeds=np.array(seeds[train:]), cold=data["cold"][train:], Q=data["Q"][train:])
    for mode in str(modes).split(","):
        stats, warm, sur, q_end = WS.warm_vs_cold(model, scales, cases[train:], data["Q"][train:],
                                                  data["cold"][train:], max_steps=max_steps, log=log,
                                                  pred=pred, mode=mode)
        # lattice updates warm / cold (all channels have nx x ny nodes): over the seeds steady both
        # ways, and over all seeds with a failed warm run charged max_steps
        cold = np.asarray(data["cold"][train:], np.float64)
        w = np.asarray(warm, np.float64)
        both = w >= 0
        stats["updates_ratio_steady_both"] = float(w[both].sum() / cold[both].sum()) if both.any() else None
        stats["updates_ratio_all_seeds"] = float(np.where(both, w, max_steps).sum() / cold.sum())
        res["results"].append(stats)
        per_seed.update({f"warm_{mode}": warm, f"surrogate_{mode}": sur, f"Q_end_{mode}": q_end})
    if out:
        os.makedirs(out, exist_ok=True)
        np.save(os.path.join(out, "params.npy"), model.get_params())
        np.savez(os.path.join(out, "per_seed.npz"), **per_seed)
        json.dump({**res, "losses": losses}, open(os.path.join(out, "warm_start.json"), "w"), indent=1)
    return res


SWEEP_HP, SWEEP_WN = 256, 256     # padded height and window width of the sweep's network


def _sweep_windows(c, hp: int = SWEEP_HP, wn: int = SWEEP_WN):
    """Network inputs for one channel of uneven size: windows of wn columns at a
    stride of wn / 2 (the channel is periodic in x, so they wrap), rows padded to
    hp with solid nodes; each window's middle wn / 2 columns are kept."""
    from . import warmstart as WS
    ny, nx = c.solid.shape
    half = wn // 2
    starts = [k * half - wn // 4 for k in range((nx + half - 1) // half)]
    X = np.zeros((len(starts), 3, hp, wn), np.float32)
    X[:, 0] = 1.0
    cols = [np.arange(s0, s0 + wn) % nx for s0 in starts]
    for k, cc in enumerate(cols):
        X[k, 0, :ny] = c.solid[:, cc]
    X[:, 1] = c.params.f_elec / WS.F_SCALE
    X[:, 2] = (c.meta["G"] - WS.G_MID) / WS.G_HALF
    return X, starts


def sweep_warm(n=256, train=1024, epochs=10, batch=32, bf16=1, chans="32,64,128,128", max_steps=700_000,
               data_max_steps=400_000, seed=0, train_seed=1, check_every=200, window=2000, rtol=None,
               storage=0):
    """Learned warm start of the batched sweep (the 256-channel table of uneven
    widths 32-256 and lengths 512-4096), FP32 storage with the plain steady rule
    (rtol 1e-8), or FP16 with stochastic rounding and the averaged rule of
    sweep_steady (rtol 1e-5).

    Training data: ``train`` channels drawn from the same distribution as the
    table (seed ``train_seed``, a different stream) but 256 columns long, run
    cold to steady flux; network inputs and targets padded to 256 rows with
    solid nodes (outside the fluid mask of the loss).  The table's channels are
    predicted in overlapping 256-column windows (middle halves kept) and seeded
    with the predicted velocity on the cold start's density ("flow" mode), then
    run to steady flux in one batch with the same rule as the cold batch, which
    this experiment also runs.  Reported: lattice updates warm and cold, and how
    many warm channels settle within 1e-4 of their cold flux."""
    import torch

    from . import net, warmstart as WS

    def log(msg):
        print(f"# {msg}", flush=True)

    storage = int(storage)
    rounding = 1 if storage else 0
    average = storage != 0
    if rtol is None:
        rtol = 1e-5 if average else 1e-8

    def to_steady(cases, steps):
        b = lbm.Batch(cases)
        b.autotune(reps=3)
        t0 = time.perf_counter()
        res = run_to_steady(b, check_every=check_every, window=window, rtol=rtol, max_steps=steps,
                            log=log, log_every=20_000, average=average)
        return b, res, time.perf_counter() - t0

    chans = tuple(int(c) for c in str(chans).split(","))
    hp, wn = SWEEP_HP, SWEEP_WN
    # ---- training data
    rows = I.sweep_table(train, train_seed)
    tcases = []
    for r in rows:
        c = I.sweep_case(dict(r, nx=wn), storage=storage, rounding=rounding)
        c.meta["G"] = r["G"]
        tcases.append(c)
    log(f"training data: {train} channels {wn} x 32..256, cold to steady flux")
    b, res, wall_data = to_steady(tcases, data_max_steps)
    X = np.zeros((train, 3, hp, wn), np.float32)
    T = np.zeros((train, 3, hp, wn), np.float32)
    fluid = np.zeros((train, hp, wn), np.uint8)
    for i, c in enumerate(tcases):
        ny = c.solid.shape[0]
        X[i, 0] = 1.0
        X[i, 0, :ny] = c.solid
        X[i, 1] = c.params.f_elec / WS.F_SCALE
        X[i, 2] = (c.meta["G"] - WS.G_MID) / WS.G_HALF
        T[i, :, :ny] = b.moments_device(i).cpu().numpy()
        fluid[i, :ny] = c.solid == 0
    del b
    log(f"training data ready: {int(res.converged.sum())} of {train} converged, {wall_data:.0f} s")
    scales = WS.Scales.fit(T, fluid)
    Tn = (T - scales.mean.reshape(1, 3, 1, 1)) / scales.std.reshape(1, 3, 1, 1) * fluid[:, None]
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(Tn.astype(np.float32)).cuda()
    Fd = torch.from_numpy(fluid).cuda()
    model = net.Net(hp, wn, batch, chans=chans, act_bf16=bool(int(bf16)))
    model.set_params(net.he_init(net.layer_shapes(chans=chans), seed))
    t0 = time.perf_counter()
    losses = WS.train(model, Xd, Td, Fd, epochs, batch, 1e-3, 1e-5, seed, log=log, log_every=100)
    train_s = time.perf_counter() - t0
    del Xd, Td, Fd
    # ---- the table: cold
    table = I.sweep_table(n, seed)
    cold_cases = []
    for r in table:
        c = I.sweep_case(r, storage=storage, rounding=rounding)
        c.meta["G"] = r["G"]
        cold_cases.append(c)
    log(f"cold batch: {n} channels")
    b, cold, wall_cold = to_steady(cold_cases, max_steps)
    del b
    # ---- predictions and the warm batch
    t0 = time.perf_counter()
    warm_cases, used = [], 0
    for c in cold_cases:
        ny, nx = c.solid.shape
        Xw, starts = _sweep_windows(c, hp, wn)
        pred = WS.predict(model, torch.from_numpy(Xw).cuda(), scales).cpu().numpy()
        full = np.zeros((3, ny, nx), np.float32)
        for k, s0 in enumerate(starts):
            cc = np.arange(s0 + wn // 4, s0 + 3 * wn // 4) % nx
            full[:, :, cc] = pred[k, :, :ny, wn // 4:3 * wn // 4]
        fields = WS.warm_fields(full, c.solid, c.meta["G"], float(c.rho[c.solid == 0].sum()), mode="flow",
                                rho_cold=c.rho)
        if fields is None:
            warm_cases.append(c)
            continue
        used += 1
        w = I.Case(c.params, c.solid, c.rho, fields[1].astype(np.float64), fields[2].astype(np.float64),
                   name=c.name, meta=dict(c.meta))
        warm_cases.append(w)
    predict_s = time.perf_counter() - t0
    log(f"warm batch: {used} of {n} channels seeded from the prediction ({predict_s:.1f} s)")
    b, warm, wall_warm = to_steady(warm_cases, max_steps)
    del b
    dq = np.abs(warm.Q - cold.Q) / np.abs(cold.Q)
    both = warm.converged & cold.converged
    nodes = np.array([c.params.nx * c.params.ny for c in cold_cases], np.float64)
    return {"experiment": "sweep_warm", "channels": n, "train_channels": train, "train_shape": [hp, wn],
            "epochs": epochs, "train_seconds": train_s, "data_seconds": wall_data,
            "data_converged": int(res.converged.sum()), "final_train_loss": losses[-1][1],
            "storage": storage, "steady_rule": {"rtol": rtol, "averaged": average, "window": window},
            "cold": {"converged": int(cold.converged.sum()), "lattice_updates": cold.node_updates,
                     "wall_seconds": wall_cold, "steps_median": float(np.median(cold.steps))},
            "warm": {"seeded": used, "converged": int(warm.converged.sum()),
                     "lattice_updates": warm.node_updates, "wall_seconds": wall_warm + predict_s,
                     "steps_median": float(np.median(warm.steps))},
            "lattice_updates_warm_over_cold": warm.node_updates / cold.node_updates,
            "lattice_updates_warm_over_cold_both_converged":
                float((nodes * warm.steps)[both].sum() / (nodes * cold.steps)[both].sum()) if both.any() else None,
            "within_1e-4_of_cold": int((dq[both] <= 1e-4).sum()), "both_converged": int(both.sum()),
            "flux_dev_median": float(np.median(dq[both])) if both.any() else None,
            "flux_dev_max": float(dq[both].max()) if both.any() else None}


def warm_detect(train=2048, val=256, test=64, nx=256, ny=64, epochs=10, batch=32, bf16=1,
                chans="32,64,128,128", max_steps=100_000, seed=0, out="", t_cold="0,500,1000,2000,4000"):
    """Learned warm start that needs no cold reference: warm runs settle by their
    own flux rule and are checked against the prediction they started from; a
    channel judged to have settled on another steady branch restarts cold in
    the same batch (warmstart.warm_with_fallback).  The two margins of the
    check are calibrated on ``val`` held-out seeds (warm runs accepted
    unconditionally, the cold reference telling which settled on its branch);
    the ``test`` seeds are then run with the check, and only the evaluation
    uses the cold reference: failures caught, missed, false alarms, and the
    lattice updates of the warm runs (fallbacks included) against the cold
    runs, both to their own steady rule.  ``t_cold`` lists the cold prefixes
    (steps run cold before the prediction's velocity is seeded) tried on the
    validation seeds; the one with the fewest lattice updates is used."""
    import torch

    from . import net, warmstart as WS

    def log(msg):
        print(f"# {msg}", flush=True)

    chans = tuple(int(c) for c in str(chans).split(","))
    n_all = train + val + test
    cases = [I.warm_case(s, nx=nx, ny=ny) for s in range(n_all)]
    log(f"{n_all} channels {nx}x{ny}: steady states (cold starts)")
    t0 = time.perf_counter()
    data = WS.steady_states(cases, max_steps=max_steps, log=log)
    X, fluid = WS.features(cases)
    T = data["T"]
    scales = WS.Scales.fit(T[:train], fluid[:train])
    Tn = (T - scales.mean.reshape(1, 3, 1, 1)) / scales.std.reshape(1, 3, 1, 1)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(Tn.astype(np.float32)).cuda()
    Fd = torch.from_numpy(fluid).cuda()
    model = net.Net(ny, nx, batch, chans=chans, act_bf16=bool(int(bf16)))
    model.set_params(net.he_init(net.layer_shapes(chans=chans), seed))
    log(f"training: {model.n_params} parameters, {epochs} epochs of {train // batch} steps")
    WS.train(model, Xd[:train], Td[:train], Fd[:train], epochs, batch, 1e-3, 1e-5, seed, log=None)
    Q_inf = np.asarray(data["Q"])
    cold_steps = np.asarray(data["steps"], np.int64)

    def on_branch(q, idx):
        return np.abs(q - Q_inf[idx]) <= 1e-4 * np.abs(Q_inf[idx])

    # calibration on the validation seeds, every warm run accepted: the cold prefix
    # (the fewest steps with the fewest off-branch warm runs) and the flux margin
    # (99th percentile of the on-branch runs' deviation from their seeded flux)
    vi = np.arange(train, train + val)
    vcases = [cases[i] for i in vi]
    calib = []
    for tc in (int(v) for v in str(t_cold).split(",")):
        rv = WS.warm_with_fallback(model, scales, vcases, q_margin=np.inf, phase_margin=1 << 30,
                                   max_steps=max_steps, t_cold=tc)
        good = on_branch(rv["Q_warm"], vi)
        upd = float(np.where(good, rv["steps"], max_steps).sum() / cold_steps[vi].sum())
        calib.append(dict(t_cold=tc, off_branch=int((~good).sum()), updates_over_cold=upd, run=rv, good=good))
        log(f"validation, cold prefix {tc}: {int((~good).sum())} of {val} warm runs off the cold branch, "
            f"updates warm / cold {upd:.3f} (off-branch runs charged {max_steps} steps)")
    best = min(calib, key=lambda c: (c["updates_over_cold"], c["t_cold"]))
    tc_best = best["t_cold"]
    rv, good = best["run"], best["good"]
    qdev = np.abs(rv["Q_warm"] - rv["Q_pred"]) / np.abs(rv["Q_pred"])
    q_margin = float(np.percentile(qdev[good], 99)) if good.any() else 0.02
    phase_margin = 1 << 30            # the phase signal does not separate branches (0 on every run)
    log(f"chosen cold prefix {tc_best} steps; flux margin {q_margin:.4f}")
    # test seeds with the check and the cold fallback
    ti = np.arange(train + val, n_all)
    rt = WS.warm_with_fallback(model, scales, [cases[i] for i in ti], q_margin=q_margin,
                               phase_margin=phase_margin, max_steps=max_steps, t_cold=tc_best)
    warm_good = on_branch(rt["Q_warm"], ti)
    final_good = on_branch(rt["Q"], ti)
    caught = int((rt["flagged"] & ~warm_good).sum())
    missed = int((~rt["flagged"] & ~final_good).sum())
    false_alarms = int((rt["flagged"] & warm_good).sum())
    wrong_warm = int((~warm_good).sum())
    nodes = float(nx * ny)
    res = {"experiment": "warm_detect", "nx": nx, "ny": ny, "train": train, "val": val, "test": test,
           "epochs": epochs, "t_cold": tc_best, "q_margin": q_margin,
           "calibration": [{k: v for k, v in c.items() if k not in ("run", "good")} for c in calib],
           "val_on_branch": int(good.sum()),
           "test_warm_off_branch": wrong_warm, "caught": caught, "missed": missed,
           "false_alarms": false_alarms, "flagged": int(rt["flagged"].sum()),
           "final_on_branch": int(final_good.sum()),
           "updates_warm_with_fallback_over_cold": float(rt["steps"].sum() / cold_steps[ti].sum()),
           "median_speedup": float(np.median(cold_steps[ti] / np.maximum(rt["steps"], 100))),
           "wall_seconds": time.perf_counter() - t0}
    log("warm detect: " + json.dumps(res))
    if out:
        import os
        os.makedirs(out, exist_ok=True)
        per = {"val": {k: np.asarray(v).tolist() for k, v in rv.items()},
               "test": {k: np.asarray(v).tolist() for k, v in rt.items()},
               "Q_inf_val": Q_inf[vi].tolist(), "Q_inf_test": Q_inf[ti].tolist(),
               "cold_steps_val": cold_steps[vi].tolist(), "cold_steps_test": cold_steps[ti].tolist()}
        json.dump({**res, "per_seed": per}, open(os.path.join(out, "warm_detect.json"), "w"))
    return res


def paper_droplet(seed=0, gc=3e-4, t_attract=10_000, t_release=20_000, t_field=10_000,
                  fs="0,0.03,0.06,0.09,0.12,0.15", nx=100, ny=50):
    """The paper's droplet run on the GPU (reading R29 of eq. (4), inputs.paper_params):
    a homogeneous fluid of density 0.85 in a 100 x 50 box gathered into one
    droplet in the middle of the substrate by an artificial attraction of
    magnitude gc (t_attract steps), released (t_release steps), then the
    electric force f on the conductive single layer next to the substrate
    for t_field steps from the released state, for every f in fs.
    Returns the released droplet's contact angle, the density of the single
    layer next to the substrate with its conductive interval [x1, x2] (the
    paper's density figure), and theta and cos(theta) - cos(theta_0) per f
    with their linear fit (the paper's eq. (9) figure)."""
    import torch

    from . import measure

    c = I.paper_droplet_case(seed, nx=nx, ny=ny)
    p, s = c.params, c.solid
    fl = s == 0
    t0 = time.perf_counter()
    sim = lbm.from_case(c)
    acc = torch.from_numpy(I.attraction_field(nx, ny, gc, s)).cuda()
    sim.set_accel_field(acc)
    sim.step(t_attract)
    sim.set_accel_field(None)
    sim.step(t_release)
    rho = sim.moments()[0].astype(np.float64)
    theta0, (xc, yc, R) = measure.contact_angle(rho, fl, y_max=ny - 4)
    row = rho[1]
    cond = np.nonzero(row >= p.rho_c)[0]
    state = sim.save_state()
    out = {"experiment": "paper_droplet", "box": [nx, ny], "seed": seed, "attraction": gc,
           "t_attract": t_attract, "t_release": t_release, "t_field": t_field,
           "theta0_deg": float(np.degrees(theta0)), "center": [float(xc), float(yc)], "radius": R,
           "layer_rho": [round(float(v), 5) for v in row],
           "x1": int(cond[0]) if len(cond) else None, "x2": int(cond[-1]) if len(cond) else None,
           "rho_range": [float(rho[fl].min()), float(rho[fl].max())], "fig3": []}
    cos0 = np.cos(theta0)
    for fe in (float(v) for v in str(fs).split(",")):
        sim.load_state(state)
        sim.set_forces(fe, 0.0, 0.0)
        sim.step(t_field)
        r = sim.moments()[0].astype(np.float64)
        th, _ = measure.contact_angle(r, fl, y_max=ny - 4)
        out["fig3"].append({"f": fe, "theta_deg": float(np.degrees(th)), "dcos": float(np.cos(th) - cos0),
                            "conductive_nodes": int((r[1] >= p.rho_c).sum())})
    f_ = np.array([e["f"] for e in out["fig3"]])
    d = np.array([e["dcos"] for e in out["fig3"]])
    if len(f_) > 1:
        A = np.stack([f_, np.ones_like(f_)], 1)
        (slope, b), *_ = np.linalg.lstsq(A, d, rcond=None)
        pred = A @ [slope, b]
        out["fit"] = {"slope": float(slope), "intercept": float(b),
                      "r2": float(1 - ((d - pred) ** 2).sum() / max(((d - d.mean()) ** 2).sum(), 1e-300))}
    out["wall_seconds"] = time.perf_counter() - t0
    return out


def _kwargs(items):
    kw = {}
    for it in items:
        k, v = it.split("=", 1)
        try:
            kw[k] = int(v)
        except ValueError:
            try:
                kw[k] = float(v)
            except ValueError:
                kw[k] = v
    return kw


def main(argv):
    name = argv[1] if len(argv) > 1 else "flux_vs_field"
    fn = {"flux_vs_field": flux_vs_field, "sweep_throughput": sweep_throughput,
          "sweep_steady": sweep_steady, "warm_start": warm_start, "channel_study": channel_study,
          "small_configs": small_configs, "net_throughput": net_throughput, "warm_detect": warm_detect,
          "paper_droplet": paper_droplet, "sweep_warm": sweep_warm}[name]
    print(json.dumps(fn(**_kwargs(argv[2:]))), flush=True)


if __name__ == "__main__":
    main(sys.argv)
