"""Experiments of the paper run on the GPU library (no oracle involved).

  flux_vs_field   Q/Q0 against the electric force f in a rough-wall channel
                  (the paper's Fig. 8 experiment; every f is one channel of a
                  batch, all advanced together to steady flux).
  sweep_throughput aggregate MLUPS of the batched engine on the 256-channel
                  sweep table (uneven widths, lengths, roughness, f and G).

Run as ``python -m paper_0708_4182_amd.experiments <name>``; prints JSON.
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


def sweep_throughput(n=256, seed=0, storage=1, steps=60, warmup=20, graph=10, tune=True):
    import torch
    rows = I.sweep_table(n, seed)
    cases = [I.sweep_case(r, storage=storage) for r in rows]
    nodes = sum(c.params.nx * c.params.ny for c in cases)
    fluid = sum(int((c.solid == 0).sum()) for c in cases)
    b = lbm.Batch(cases)
    tile = None
    if tune:
        bx, r, us = b.autotune(reps=3)
        tile = [bx, r]
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
            "storage": storage, "tile": tile, "graph_steps": graph, "ms_per_step": ms,
            "mlups": nodes / (ms * 1e-3) / 1e6,
            "achieved_GBs": 18 * es * fluid / (ms * 1e-3) / 1e9}


def main(argv):
    name = argv[1] if len(argv) > 1 else "flux_vs_field"
    fn = {"flux_vs_field": flux_vs_field, "sweep_throughput": sweep_throughput}[name]
    print(json.dumps(fn()), flush=True)


if __name__ == "__main__":
    main(sys.argv)
