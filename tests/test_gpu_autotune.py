"""Autotuner on the GPU: the particle pass's launch shape, the cell-sort period of
plain PIC runs and the Newton iterations per fine step (parity-gated)."""
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
    """Different tiles and grids give the same charge and the same macro step bit
    for bit."""
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
    # every deposit and snapshot sum is an integer sum: the same bits everywhere
    assert all(np.array_equal(charges[0], q) for q in charges[1:])
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


def iaw_coarse(E, specs):
    ctx = E.Context(E.ConfigSpec(specs))
    for r, sp in enumerate(specs):
        n0, u0 = synth.iaw_profile(sp.n_cells, sp.length)
        E.efpi_load_profile(ctx.ctx, r, torch.as_tensor(n0, device="cuda"),
                            torch.as_tensor(u0, device="cuda"), 70 + r)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 30, cold=True)
    c = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c)
    E.efpi_sync(ctx.ctx)
    ctx.close()
    return c


def test_sort_period_tuner():
    E = lib()
    from paper_1610_01071_amd import autotune
    sp = E.ReplicaSpec(1024, 1024.0, ppc=100, haar_levels=2, vth=0.316)
    c0 = iaw_coarse(E, [sp])
    period, table = autotune.sort_period(sp, c0, 7, periods=(10, 50, 0), steps=120, tile=1024)
    assert [t["sort_period"] for t in table] == [10, 50, 0]
    assert period == min(table, key=lambda t: t["ms"])["sort_period"]
    assert all(t["device_status"] == 0 for t in table)


def test_sort_period_does_not_change_a_plain_run():
    """A sort permutes the ions; each push is per ion and the deposit an integer
    sum, so plain PIC runs with and without sorts end in the same coarse state."""
    E = lib()
    sp = E.ReplicaSpec(1024, 1024.0, ppc=100, haar_levels=2, vth=0.316)
    c0 = iaw_coarse(E, [sp])
    outs = []
    for period in (10, 0):
        ctx = E.Context(E.ConfigSpec([sp], tile=1024, flags=E.FLAG_SORT_BUFFER))
        E.efpi_lift(ctx.ctx, c0, [9])
        done = 0
        while done < 60:
            k = 60 - done if period == 0 else min(period, 60 - done)
            E.efpi_pic_burst(ctx.ctx, k, False)
            done += k
            if done < 60:
                E.efpi_sort(ctx.ctx)
        c = ctx.new_coarse()
        E.efpi_restrict_state(ctx.ctx, c)
        E.efpi_sync(ctx.ctx)
        outs.append(c.cpu().numpy())
        ctx.close()
    assert np.array_equal(outs[0], outs[1])


def test_newton_iterations_tuner():
    E = lib()
    from paper_1610_01071_amd import autotune
    specs = specs_small(E)[:2]
    c0 = iaw_coarse(E, specs)
    iters, table = autotune.newton_iterations(specs, c0, [1, 2], candidates=(1, 2, 3),
                                              reference=6, eps_max=1e-3, steps=1, tile=1024)
    assert [t["newton_iters"] for t in table] == [1, 2, 3]
    by = {t["newton_iters"]: t for t in table}
    # three iterations from the burst's warm start are within 1e-3 of six
    assert by[3]["admissible"] and by[3]["eps_vs_reference"] <= 1e-3
    assert iters in by and by[iters]["admissible"]
    assert by[iters]["ms_per_step"] == min(t["ms_per_step"] for t in table if t["admissible"])
