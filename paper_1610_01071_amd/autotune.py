"""Autotuner of the burst: launch shape of the particle pass (tile size and grid),
the cell-sort period of long plain-PIC runs, and the Newton iterations per fine
step.

For a list of replicas, every (tile, grid_blocks) candidate gets its own
library context; each runs warm-up macro steps and then timed macro steps
(HIP events on the context's stream) from the same coarse state.  The fastest
candidate is returned and, when a cache file is given, stored as JSON keyed by
the device name and the replica sizes, so later runs reuse it.  Tile and grid
never change what is computed: every deposit and snapshot sum is an integer
sum, so all candidates give the same bits.

The sort period S (plain PIC: a stable cell sort every S steps keeps each wave's
ions within its LDS windows) trades the sort's cost against the particle pass's
slowdown as the cell order decays; candidates are timed on a plain run.  The
Newton iteration count is parity-gated: a count is admissible only when its
macro step stays within a stated eps (eq. 4.2) of the same step with more
iterations and raises no Newton flag; the fastest admissible count is returned.
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


def sort_period(spec, coarse, shift, periods=(10, 25, 50, 100, 200, 0), steps=200, newton_iters=2,
                tile=2048):
    """Fastest cell-sort period for `steps` plain PIC steps of one replica lifted from
    `coarse` (0: never sort).  Returns (period, table of ms per run)."""
    table = []
    for period in periods:
        ctx = E.Context(E.ConfigSpec([spec], newton_iters=newton_iters, newton_iters_start=4,
                                     tile=tile, flags=E.FLAG_SORT_BUFFER))
        try:
            def run():
                E.efpi_lift(ctx.ctx, coarse, [shift])
                done = 0
                while done < steps:
                    k = steps - done if period == 0 else min(period, steps - done)
                    E.efpi_pic_burst(ctx.ctx, k, False)
                    done += k
                    if done < steps:
                        E.efpi_sort(ctx.ctx)

            run()  # warm-up
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            run()
            e1.record()
            torch.cuda.synchronize()
            bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
            table.append({"sort_period": period, "ms": e0.elapsed_time(e1), "device_status": bits})
        finally:
            ctx.close()
    best = min(table, key=lambda t: t["ms"])
    return best["sort_period"], table


def newton_iterations(specs, coarse, shifts, candidates=(1, 2, 3), reference=4, eps_max=1e-4,
                      steps=3, tile=4096, grid_blocks=0):
    """Fewest-cost Newton iterations per fine step whose macro step from `coarse`
    stays within eps_max (eq. 4.2, every replica's density and momentum) of the
    step with `reference` iterations and sets no Newton flag.  Returns
    (iterations, table)."""
    def run(iters, timed_steps):
        ctx = E.Context(E.ConfigSpec(list(specs), newton_iters=iters, newton_iters_start=4,
                                     tile=tile, grid_blocks=grid_blocks))
        try:
            out = torch.empty_like(coarse)
            E.efpi_macro_step(ctx.ctx, coarse, out, shifts)
            bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
            first = out.clone()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(timed_steps):
                E.efpi_macro_step(ctx.ctx, coarse, out, shifts)
            e1.record()
            torch.cuda.synchronize()
            return first, bits, e0.elapsed_time(e1) / max(timed_steps, 1)
        finally:
            ctx.close()

    ref, _, _ = run(reference, 0)
    table = []
    for iters in candidates:
        got, bits, ms = run(iters, steps)
        eps = 0.0
        o = 0
        out = torch.zeros(1, dtype=torch.float64, device=coarse.device)
        for r in specs:
            for m in range(2):
                sl = slice(o + m * r.n_coarse, o + (m + 1) * r.n_coarse)
                E.efpi_rel_l2(got[sl], ref[sl], out)
                eps = max(eps, float(out.item()))
            o += 2 * r.n_coarse
        ok = eps <= eps_max and not (bits & (E.DEV_NEWTON | E.DEV_NAN))
        table.append({"newton_iters": iters, "eps_vs_reference": eps, "device_status": bits,
                      "admissible": ok, "ms_per_step": ms})
    good = [t for t in table if t["admissible"]]
    best = min(good, key=lambda t: t["ms_per_step"]) if good else None
    return (best["newton_iters"] if best else reference), table
