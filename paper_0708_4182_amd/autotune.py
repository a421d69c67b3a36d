"""Tile autotuning with a JSON cache keyed by GPU architecture.

The timing itself runs in the library (lbm_autotune: candidate tiles launched
on the device, state untouched); this module only remembers the winner per
(architecture, storage, lattice size) so later runs skip the search.
"""
from __future__ import annotations

import json
import os
import tempfile

CACHE = os.environ.get("LBM_TILE_CACHE") or os.path.join(
    os.path.expanduser("~"), ".cache", "lbm_mi355x", "tiles.json")


def _arch(sim) -> str:
    props = sim.torch.cuda.get_device_properties(sim.device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(path: str, data: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=os.path.dirname(path), suffix=".tmp")
        with os.fdopen(fd, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs a re-tune next time


def tune(sim, reps: int = 5, cache: str | None = CACHE, refresh: bool = False):
    """Set the fastest kernel and tile on ``sim``; returns
    (kernel, block_x, rows, us_per_step, cached)."""
    key = f"{_arch(sim)}/storage{int(sim.params.storage)}/{sim.nx}x{sim.ny}"
    data = _load(cache) if cache else {}
    entry = data.get(key)
    if not refresh and isinstance(entry, list) and len(entry) == 4:
        kernel, bx, rows, us = entry
        sim.set_kernel(str(kernel))
        sim.set_tile(int(bx), int(rows))
        return str(kernel), int(bx), int(rows), float(us), True
    bx, rows, us = sim.autotune(reps)
    kernel = sim.tile()[0]
    if cache:
        data = _load(cache)
        data[key] = [kernel, bx, rows, us]
        _save(cache, data)
    return kernel, bx, rows, us, False
