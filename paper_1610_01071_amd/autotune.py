"""Launch-shape autotuner for the particle pass (tile size and persistent grid).

For a list of replicas, every candidate (tile, grid_blocks) gets its own
library context; each runs warm-up macro steps and then timed macro steps
(HIP events on the context's stream) from the same coarse state.  The fastest
candidate is returned and, when a cache file is given, stored as JSON keyed by
the device name and the replica sizes, so later runs reuse it.  Every
candidate computes the same result (tile and grid only change the order in
which work items are visited and which integer sums a workgroup merges), so
choosing one never changes what is computed beyond rounding of FP32 partial
sums inside the restriction merge.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass

import numpy as np
import torch

from . import efpi as E

TILES = (1024, 2048, 3072, 4096, 8192)
GRIDS = (1024, 2048, 4096, 1 << 20)  # the last: one workgroup per work item


@dataclass
class Choice:
    tile: int
    grid_blocks: int
    ms_per_step: float
    table: list


def cache_key(specs) -> str:
    dev = torch.cuda.get_device_name(0) if torch.cuda.is_available() else "none"
    sizes = ";".join(f"{r.n_cells}x{r.ppc}x{r.burst_steps}x{r.bc}" for r in specs)
    return f"{dev}|{sizes}"


def load_cache(path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def save_cache(path, cache):
    if not path:
        return
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def uniform_coarse(specs, device="cuda"):
    """Coarse state of a uniform plasma (n = 1, u = 0) for every replica."""
    parts = []
    for r in specs:
        scale = 2.0 ** (r.haar_levels / 2.0)
        parts.append(np.stack([np.full(r.n_coarse, scale), np.zeros(r.n_coarse)]).ravel())
    return torch.as_tensor(np.concatenate(parts), dtype=torch.float64, device=device)


def time_candidate(specs, tile, grid_blocks, steps, warmup, newton_iters=2, flags=0):
    ctx = E.Context(E.ConfigSpec(list(specs), newton_iters=newton_iters, newton_iters_start=4,
                                 tile=tile, grid_blocks=grid_blocks, flags=flags))
    try:
        a = uniform_coarse(specs)
        b = torch.empty_like(a)
        shifts = [1 + r for r in range(len(specs))]
        for _ in range(warmup):
            E.efpi_macro_step(ctx.ctx, a, b, shifts)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            E.efpi_macro_step(ctx.ctx, a, b, shifts)
        e1.record()
        torch.cuda.synchronize()
        E.efpi_sync(ctx.ctx, raise_on_error=False)
        return e0.elapsed_time(e1) / steps
    finally:
        ctx.close()


def autotune(specs, tiles=TILES, grids=GRIDS, steps=3, warmup=1, cache_path=None,
             newton_iters=2) -> Choice:
    """Fastest (tile, grid_blocks) for the replicas in `specs`."""
    cache = load_cache(cache_path)
    key = cache_key(specs)
    if key in cache:
        c = cache[key]
        return Choice(c["tile"], c["grid_blocks"], c["ms_per_step"], c.get("table", []))
    table = []
    for tile in tiles:
        for grid in grids:
            ms = time_candidate(specs, tile, grid, steps, warmup, newton_iters)
            table.append({"tile": tile, "grid_blocks": grid, "ms_per_step": ms})
    best = min(table, key=lambda t: t["ms_per_step"])
    choice = Choice(best["tile"], best["grid_blocks"], best["ms_per_step"], table)
    cache[key] = {"tile": choice.tile, "grid_blocks": choice.grid_blocks,
                  "ms_per_step": choice.ms_per_step, "table": table}
    save_cache(cache_path, cache)
    return choice
