#!/usr/bin/env python3
"""Throughput of the fused EWOD Shan-Chen D2Q9 step on one MI355X.

Workload: one rough-wall channel of 8192 x 2048 nodes with random steps on both
walls (height 2..8, pitch 16..64, width pitch/4), liquid with a vapour layer at
the walls, G = -5, tau = 1, electric force 1e-3 on the near-wall liquid and a
driving acceleration of 1e-6 along x (synthetic, seed 0).

A timed step is one launch of the fused collide-stream kernel over the whole
lattice; the timed region ends with one FP64 flux/mass reduction (the monitor
a steady-flux run takes every few hundred steps).  Inputs are resident in HBM
before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "MLUPS + % HBM roofline; steady-flux lattice updates, warm-start vs plain"
HBM_PEAK_GBS = 8000.0
STORAGES = {"f32": 0, "f16": 1, "bf16": 2}
# extra lines: name -> (storage, collision, rounding); collision 1 is the TRT operator with Guo
# forcing, rounding 1 the stochastic rounding of 16-bit stores
VARIANTS = {"f16": (1, 0, 0), "bf16": (2, 0, 0), "f32_trt": (0, 1, 0), "f32_mrt": (0, 2, 0), "f16_sr": (1, 0, 1),
            "bf16_sr": (2, 0, 1)}
ELEM_BYTES = {0: 4, 1: 2, 2: 2}
STEPS_PER_LAUNCH = {"two": 2, "three": 3}     # kernels that advance more than one time step per launch
KERNEL_SRC = os.path.join(ROOT, "paper_0708_4182_amd", "csrc", "lbm_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def kernel_sha() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


KERNEL_NAMES = {
    "fused": "k_step (fused pull-stream + bounce-back + Shan-Chen/EWOD forces + BGK, one column per thread)",
    "wide2": "k_step_wide<2> (the fused step, two adjacent columns per thread)",
    "wide4": "k_step_wide<4> (the fused step, four adjacent columns per thread)",
    "split": "k_step_split (producer wave streams rows into LDS; compute waves collide and store)",
    "fused8": "k_step8 (the fused step compiled for 8 waves per SIMD, one column per thread)",
    "two": "k_stepk<..., 2> (two time steps per launch, the first step's results in LDS: temporal blocking)",
    "three": "k_stepk<..., 3> (three time steps per launch, intermediate results in LDS: temporal blocking)",
}


def measured_traffic(storage_name: str, tile):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    if they were taken on a different kernel source, kernel or tile."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    recs = t.get(storage_name) or []
    for e in [recs] if isinstance(recs, dict) else recs:
        if isinstance(e, dict) and e.get("kernel_sha") == kernel_sha() and list(e.get("tile", [])) == list(tile):
            return e.get("bytes_per_launch")
    return None


def time_storage(case, storage, steps, warmup, tile, collision=0, rounding=0):
    import torch
    from paper_0708_4182_amd import lbm

    from paper_0708_4182_amd import autotune

    c = case.params.replace(storage=storage, collision=collision, rounding=rounding)
    sim = lbm.Simulation(c, case.solid, case.rho, case.ux, case.uy)
    if tile:
        kernel, bx, rows = tile
        sim.set_kernel(kernel)
        sim.set_tile(bx, rows)
        chosen = [bx, rows, kernel]
    else:
        kernel, bx, rows, us, cached = autotune.tune(sim, reps=20, cache=None)
        chosen = [bx, rows, kernel]
    sim.step(warmup)
    sim.flux()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    with torch.cuda.stream(sim.stream):
        t0 = time.perf_counter()
        ev[0].record(sim.stream)
        sim.step(steps)
        ev[1].record(sim.stream)
        Q, M = sim.flux()            # synchronizes
        ev[2].record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = ev[0].elapsed_time(ev[1]) / steps
    total_ms = ev[0].elapsed_time(ev[2])
    del sim
    torch.cuda.empty_cache()
    return dict(step_ms=step_ms, total_ms=total_ms, wall_s=wall, Q=Q, M=M, tile=chosen)


def copy_ceiling(nbytes: int, reps: int = 20):
    """GB/s (read + write counted) of the library's one-pass non-temporal
    streaming copy (lbm_stream_copy) of a buffer the size of one population
    buffer, best over 1, 2 and 4 chunks of 16 bytes per lane: the practical
    HBM ceiling.  torch's device copy of the same buffer is reported beside it."""
    import torch
    from paper_0708_4182_amd import lbm

    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = None
    for per_lane in (1, 2, 4):
        lbm.stream_copy(b, a, per_lane)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            lbm.stream_copy(b, a, per_lane)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if best is None or ms < best[0]:
            best = (ms, per_lane)
    assert torch.equal(a, b)
    b.copy_(a)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    tms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    ms, per_lane = best
    return {"GB/s": round(2 * nbytes / (ms * 1e-3) / 1e9, 1), "bytes_copied": nbytes, "ms": round(ms, 4),
            "kernel": f"lbm_stream_copy (one pass, {per_lane} x 16 B per lane, non-temporal)",
            "torch_copy_GB/s": round(2 * nbytes / (tms * 1e-3) / 1e9, 1)}


def step_line(name: str, r: dict, nsites: int, nfluid: int) -> dict:
    """Bench line of one storage/variant run r (time_storage's result) on a
    lattice of nsites nodes, nfluid of them fluid: rate and HBM roofline."""
    s = STORAGES[name] if name in STORAGES else VARIANTS[name][0]
    # algorithmic HBM bytes of one launch: every population read once and
    # written once (18 values per fluid node); a multi-step kernel's launch
    # covers two or three time steps
    steps_per_launch = STEPS_PER_LAUNCH.get(r["tile"][2], 1)
    alg_bytes = 18 * ELEM_BYTES[s] * nfluid
    launch_ms = r["step_ms"] * steps_per_launch
    achieved = alg_bytes / (launch_ms * 1e-3) / 1e9
    traffic = measured_traffic(name, r["tile"])
    line = {
        "tile": r["tile"],
        "mlups": round(nsites / (r["step_ms"] * 1e-3) / 1e6, 1),
        "ms_per_step": round(r["step_ms"], 5),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "steps_per_launch": steps_per_launch,
                     "launch_ms": round(launch_ms, 5)},
    }
    if steps_per_launch > 1:
        # what a kernel that streams the populations once per step would need for this step rate
        eq = alg_bytes / (r["step_ms"] * 1e-3) / 1e9
        line["roofline"]["single_step_equivalent"] = {"GB/s": round(eq, 1), "frac": round(eq / HBM_PEAK_GBS, 4)}
    return line


def batch_line(bt: dict) -> dict:
    """Bench line of the sweep-table batch (experiments.sweep_throughput's
    result bt, hipGraphs of 12 steps: whole numbers of one-, two- and
    three-step launches): the roofline per launch, whose algorithmic bytes
    are those of one step, and the single-step equivalent beside it."""
    spl = {"fused": 1, "two": 2, "three": 3}[bt["kernel"]]
    per_launch = bt["achieved_GBs"] / spl
    line = {"workload": "256-channel sweep table (width 32-256, length 512-4096, "
                        "step height 0-8, f in [0,3e-3), G in [-5.5,-4.5]), FP16 storage with "
                        "stochastic rounding, steps per launch and tile autotuned (a workgroup "
                        "per tile or a persistent queue), hipGraph of 12 steps",
            "mlups": round(bt["mlups"], 1), "ms_per_step": round(bt["ms_per_step"], 4),
            "kernel": bt["kernel"], "tile": bt["tile"],
            "roofline": {"bound": "hbm", "achieved": round(per_launch, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(per_launch / HBM_PEAK_GBS, 4), "steps_per_launch": spl}}
    if spl > 1:
        line["roofline"]["single_step_equivalent"] = {
            "GB/s": round(bt["achieved_GBs"], 1), "frac": round(bt["achieved_GBs"] / HBM_PEAK_GBS, 4)}
    return line


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(steps: int):
    """The FP64 oracle on the host: single-threaded, then on all the threads its
    OpenMP loops use (OMP_NUM_THREADS, else every core); both runs step the
    same state bitwise alike.  The line's value is the all-threads rate."""
    import oracle as O
    from paper_0708_4182_amd import inputs as I

    c = I.random_channel_case(nx=512, ny=128, seed=0)
    n0 = O.threads()
    rates = {}
    try:
        for nth, nsteps in ((1, steps), (n0, 4 * steps)):
            O.threads(nth)
            f = O.init(c.params, c.solid, c.rho)
            t0 = time.perf_counter()
            O.step(c.params, c.solid, f, nsteps)
            dt = time.perf_counter() - t0
            rates[nth] = (512 * 128 * nsteps / dt / 1e6, nsteps, dt)
    finally:
        O.threads(n0)
    v, nsteps, dt = rates[n0]
    v1, steps1, dt1 = rates[1]
    return {"value": round(v, 3), "unit": "MLUPS", "cores": n0, "kind": "oracle",
            "sample": f"FP64 oracle, {n0} OpenMP threads, 512x128 instance of the same random-step "
                      f"generator (seed 0), {nsteps} steps, {dt:.1f} s",
            "single_thread": {"value": round(v1, 3), "unit": "MLUPS", "cores": 1,
                              "sample": f"the same, one thread, {steps1} steps, {dt1:.1f} s"},
            "cpu_model": cpu_model(), "cpus_visible": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--storage", default="f32", choices=sorted(STORAGES))
    ap.add_argument("--variants", default="f16,bf16,f32_trt,f32_mrt,f16_sr,bf16_sr",
                    help="other lines timed after the main one: f16, bf16 (storage), f32_trt, f32_mrt (FP32 "
                         "storage with the TRT or MRT collision and Guo forcing), f16_sr, bf16_sr (16-bit "
                         "storage with stochastic rounding); '' for none")
    ap.add_argument("--nx", type=int, default=8192)
    ap.add_argument("--ny", type=int, default=2048)
    ap.add_argument("--tile", default="auto",
                    help="[kernel:]block_x x rows, e.g. 512x64, split:128x0 or two:512x137 (rows 0 = one wave "
                         "of workgroups; kernel fused, fused8, split, wide2, wide4 or two), or 'auto'")
    ap.add_argument("--cpu-steps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-copy-ceiling", action="store_true")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the learned warm-start line (about 40 s: 2112 steady states, training, 64 seeds)")
    ap.add_argument("--no-network", action="store_true",
                    help="skip the warm-start network line (training and inference rate)")
    ap.add_argument("--no-small", action="store_true",
                    help="skip the launch-bound line (128x64 droplet, 1024x128 rough channel)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched-sweep line (256 uneven channels, FP16 storage)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "the multi-GPU halo exchange is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0708_4182_amd import inputs as I

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    tile = None
    if args.tile not in ("", "auto"):
        kernel, _, t = args.tile.rpartition(":")
        bx, rows = (int(v) for v in t.split("x"))
        tile = (kernel or "fused", bx, rows)
    case = I.random_channel_case(nx=args.nx, ny=args.ny, f_elec=1e-3, seed=0)
    nsites = args.nx * args.ny
    nfluid = int((case.solid == 0).sum())


    main_r = time_storage(case, STORAGES[args.storage], args.steps, args.warmup, tile)
    print(f"# {args.storage}: tile {main_r['tile']} {main_r['step_ms']*1e3:.1f} us/step, "
          f"Q={main_r['Q']:.6e} M={main_r['M']:.6e}",
          file=sys.stderr, flush=True)
    main_line = step_line(args.storage, main_r, nsites, nfluid)
    variants = {}
    for v in [v for v in args.variants.split(",") if v and v != args.storage]:
        st, coll, rnd = VARIANTS[v] if v in VARIANTS else (STORAGES[v], 0, 0)
        vt = tile
        if (coll or rnd) and tile and tile[0] not in ("fused", "fused8", "two", "three"):
            vt = ("fused", tile[1], tile[2])     # TRT, MRT and stochastic rounding: fused and multi-step kernels only
        r = time_storage(case, st, args.steps, args.warmup, vt, collision=coll, rounding=rnd)
        print(f"# {v}: tile {r['tile']} {r['step_ms']*1e3:.1f} us/step", file=sys.stderr, flush=True)
        variants[v] = step_line(v, r, nsites, nfluid)

    ms_per_step = main_r["total_ms"] / args.steps
    value = nsites * args.steps / (main_r["total_ms"] * 1e-3) / 1e6
    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"random-step rough channel {args.nx}x{args.ny} (step height 2-8, "
                               f"pitch 16-64), G=-5, tau=1, f_elec=1e-3, g=1e-6, seed 0",
                   "nx": args.nx, "ny": args.ny, "storage": args.storage,
                   "tile": main_r["tile"], "tile_choice": "fixed" if tile else "autotuned",
                   "fluid_nodes": nfluid},
        "roofline": main_line["roofline"],
        "kernel": KERNEL_NAMES[main_r["tile"][2]],
        "variants": variants,
    }
    if not args.no_batch:
        from paper_0708_4182_amd import experiments
        bt = experiments.sweep_throughput(graph=12)
        print(f"# batch: {bt['channels']} channels, {bt['nodes']} nodes, {bt['kernel']} tile {bt['tile']}, "
              f"{bt['ms_per_step']*1e3:.1f} us/step", file=sys.stderr, flush=True)
        out["batch"] = batch_line(bt)
    if not args.no_warm_start:
        import contextlib
        from paper_0708_4182_amd import experiments
        t0 = time.perf_counter()
        with contextlib.redirect_stdout(sys.stderr):     # the experiment's progress lines
            ws = experiments.warm_detect(train=4096, val=128, test=64, epochs=30, t_cold="0")
        out["warm_start"] = {
            "workload": "learned warm start on 256x64 channels (step height 0-8, f in [0,3e-3), G in "
                        "[-5.5,-4.5], g = 1e-6, FP32): network trained by the library's kernels on 4096 "
                        "steady states the method generates (30 epochs); 64 held-out seeds seeded from its "
                        "predicted velocity (flow mode), each run to its own steady flux (|dQ| <= 1e-8 |Q| "
                        "over 1000 steps, the cold runs' rule) with no cold reference; a settled run whose "
                        "flux departs from its seeded flux by more than a margin calibrated on 128 other "
                        "seeds restarts cold in the same batch",
            "lattice_updates_warm_over_plain": round(ws["updates_warm_with_fallback_over_cold"], 4),
            "median_speedup": round(ws["median_speedup"], 3),
            "seeds": ws["test"], "warm_off_cold_branch": ws["test_warm_off_branch"],
            "caught": ws["caught"], "missed": ws["missed"], "false_alarms": ws["false_alarms"],
            "final_within_1e-4_of_cold": ws["final_on_branch"],
            "flux_margin": round(ws["q_margin"], 4),
            "wall_seconds": round(time.perf_counter() - t0, 1),
            "note": "off-branch: the warm run settles more than 1e-4 from the cold start's steady flux; the "
                    "cold reference is used only to count caught / missed / false alarms"}
        print(f"# warm start: {out['warm_start']}", file=sys.stderr, flush=True)
    if not args.no_network:
        from paper_0708_4182_amd import experiments
        nt = experiments.net_throughput()
        print(f"# network: {nt}", file=sys.stderr, flush=True)
        out["network"] = {"workload": "warm-start encoder-decoder (channels 32/64/128/128, 15 layers), batch of 32 "
                                      "samples of 3 x 64 x 256, bf16 activations, random He-initialised weights "
                                      "and random inputs; train = forward + backward + Adam",
                          **nt,
                          "roofline": {"bound": "mfma", "achieved": nt["infer"]["tflops"], "peak": 2500.0,
                                       "unit": "TFLOP/s", "frac": round(nt["infer"]["tflops"] / 2500.0, 4),
                                       "note": "inference; the bf16 dense MFMA peak"}}
    if not args.no_small:
        from paper_0708_4182_amd import experiments
        sm = experiments.small_configs()
        print(f"# small: {sm}", file=sys.stderr, flush=True)
        out["small"] = {"workload": "launch-bound lattices, FP32, autotuned: 128x64 droplet (R = 20, f = 1e-3) "
                                    "and 1024x128 rough channel (a=8, b=4, p=32, f = 1e-3); ordinary lbm_step "
                                    "launches vs hipGraph replays of 50 steps (lbm_set_graph); no roofline "
                                    "claim (the lattices fit in cache)",
                        **sm}
    if not args.no_copy_ceiling:
        out["copy_ceiling"] = copy_ceiling(9 * nsites * ELEM_BYTES[STORAGES[args.storage]])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
