"""Autotuner of the particle pass launch shape, on the GPU."""
import json

import numpy as np
import pytest
import torch

import synth
from helpers import lib

pytestmark = pytest.mark.gpu


def specs_small(E):
    return [E.ReplicaSpec(256, 256.0, ppc=64, haar_levels=3, burst_steps=6, macro_dt=2.0),
            E.ReplicaSpec(1024, 1024.0, ppc=32, haar_levels=4, burst_steps=6, macro_dt=2.0),
            E.ReplicaSpec(2048, 2048.0, ppc=20, haar_levels=4, burst_steps=6, macro_dt=2.0)]


def test_autotune_picks_fastest_and_caches(tmp_path):
    E = lib()
    from paper_1610_01071_amd import autotune
    specs = specs_small(E)
    path = str(tmp_path / "tune.json")
    c = autotune.autotune(specs, tiles=(1024, 4096), grids=(1024, 1 << 20), steps=2, warmup=1,
                          cache_path=path)
    assert len(c.table) == 4
    assert c.ms_per_step == min(t["ms_per_step"] for t in c.table)
    assert (c.tile, c.grid_blocks) in [(t["tile"], t["grid_blocks"]) for t in c.table]
    saved = json.load(open(path))
    assert autotune.cache_key(specs) in saved
    # second call is served from the cache without timing anything
    c2 = autotune.autotune(specs, tiles=(1024,), grids=(1024,), cache_path=path)
    assert (c2.tile, c2.grid_blocks) == (c.tile, c.grid_blocks)


def test_launch_shapes_agree():
    """Different tiles and grids give the same charge bit for bit and the same
    coarse state up to FP32 rounding of the restriction's partial sums."""
    E = lib()
    specs = specs_small(E)
    outs, charges = [], []
    for tile, grid in ((1024, 1024), (4096, 1 << 20), (2048, 64)):
        ctx = E.Context(E.ConfigSpec(specs, tile=tile, grid_blocks=grid))
        for r, sp in enumerate(specs):
            n0, u0 = synth.iaw_profile(sp.n_cells, sp.length)
            E.efpi_load_profile(ctx.ctx, r, torch.as_tensor(n0, device="cuda"),
                                torch.as_tensor(u0, device="cuda"), 40 + r)
        E.efpi_deposit(ctx.ctx)
        charges.append(torch.cat([ctx.grid(r)[0] for r in range(len(specs))]).cpu().numpy())
        E.efpi_solve_field(ctx.ctx, 20, cold=True)
        a = ctx.new_coarse()
        E.efpi_restrict_state(ctx.ctx, a)
        b = ctx.new_coarse()
        E.efpi_macro_step(ctx.ctx, a, b, [3, 4, 5])
        outs.append(b.cpu().numpy())
        ctx.close()
    assert all(np.array_equal(charges[0], q) for q in charges[1:])
    for o in outs[1:]:
        assert np.sqrt(np.sum((o - outs[0]) ** 2) / np.sum(o ** 2 + outs[0] ** 2)) < 1e-5
