"""Captured macro steps (efpi_macro_step_graph) against the eager path.

Each captured graph is replayed several times, with eager library work, torch
work and stream synchronisations between the replays, and every replay's
coarse output must equal the eager macro step's bit for bit (both paths run
the same kernels with the same arguments; only the enqueueing differs).
"""
import numpy as np
import pytest
import torch

import synth
from helpers import lib

pytestmark = pytest.mark.gpu


def start(E, ctx, spec, seed):
    n0, u0 = synth.iaw_profile(spec.n_cells, spec.length)
    E.efpi_load_profile(ctx.ctx, 0, torch.as_tensor(n0, device="cuda"),
                        torch.as_tensor(u0, device="cuda"), synth.lift_shift(seed))
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 20, cold=True)
    c = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c)
    return c


@pytest.mark.parametrize("n_cells,ppc,steps,k", [(512, 100, 6, 20), (256, 64, 5, 7)])
def test_graph_replays_equal_eager(n_cells, ppc, steps, k):
    E = lib()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        spec = E.ReplicaSpec(n_cells, float(n_cells), ppc=ppc, haar_levels=4, burst_steps=k,
                             macro_dt=5.0)
        ce = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=4))
        cg = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=4))
        ae, ag = start(E, ce, spec, 3), start(E, cg, spec, 3)
        assert torch.equal(ae, ag)
        be, bg = ce.new_coarse(), cg.new_coarse()
        junk = torch.zeros(1 << 20, device="cuda")
        for i in range(steps):
            sh = [synth.lift_shift(1000 + i)]
            E.efpi_macro_step(ce.ctx, ae, be, sh)
            E.efpi_macro_step_graph(cg.ctx, ag, bg, sh)
            # eager work and synchronisation between replays
            junk.add_(1.0)
            side.synchronize()
            assert torch.equal(be, bg), f"step {i}"
            ae, be = be, ae
            ag, bg = bg, ag
        # eager library calls on the graph context keep its state consistent
        E.efpi_pic_burst(cg.ctx, 3, False)
        E.efpi_pic_burst(ce.ctx, 3, False)
        E.efpi_macro_step_graph(cg.ctx, ag, bg, [7])
        E.efpi_macro_step(ce.ctx, ae, be, [7])
        side.synchronize()
        assert torch.equal(be, bg)
        assert E.efpi_sync(cg.ctx, raise_on_error=False) == E.efpi_sync(ce.ctx, raise_on_error=False)


def test_graph_needs_a_stream():
    E = lib()
    spec = E.ReplicaSpec(64, 64.0, ppc=16, haar_levels=2, burst_steps=4, macro_dt=1.0)
    ctx = E.Context(E.ConfigSpec([spec]), stream=torch.cuda.default_stream())
    c = ctx.new_coarse()
    with pytest.raises(E.EfpiError) as ei:
        E.efpi_macro_step_graph(ctx.ctx, c, c, [1])
    assert "stream" in str(ei.value)


def test_graph_ensemble_equals_eager():
    E = lib()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        specs = [E.ReplicaSpec(256, 256.0, ppc=50, haar_levels=3, burst_steps=10, macro_dt=3.0),
                 E.ReplicaSpec(1024, 1024.0, ppc=20, haar_levels=4, burst_steps=10, macro_dt=3.0)]
        ce = E.Context(E.ConfigSpec(specs))
        cg = E.Context(E.ConfigSpec(specs))
        a = ce.new_coarse()
        for r, sp in enumerate(specs):
            n0, u0 = synth.iaw_profile(sp.n_cells, sp.length)
            for c in (ce, cg):
                E.efpi_load_profile(c.ctx, r, torch.as_tensor(n0, device="cuda"),
                                    torch.as_tensor(u0, device="cuda"), 11 + r)
        for c in (ce, cg):
            E.efpi_deposit(c.ctx)
            E.efpi_solve_field(c.ctx, 20, cold=True)
        E.efpi_restrict_state(ce.ctx, a)
        ag = a.clone()
        be, bg = ce.new_coarse(), cg.new_coarse()
        for i in range(4):
            E.efpi_macro_step(ce.ctx, a, be, [5 + i, 9 + i])
            E.efpi_macro_step_graph(cg.ctx, ag, bg, [5 + i, 9 + i])
            side.synchronize()
            assert torch.equal(be, bg)
            a, be = be, a
            ag, bg = bg, ag


def test_graph_cache_is_bounded():
    """More distinct (input, output) pairs than the cache holds: every call still
    equals the eager macro step."""
    E = lib()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        spec = E.ReplicaSpec(128, 128.0, ppc=32, haar_levels=2, burst_steps=4, macro_dt=1.0)
        ce = E.Context(E.ConfigSpec([spec]))
        cg = E.Context(E.ConfigSpec([spec]))
        a = start(E, ce, spec, 4)
        start(E, cg, spec, 4)
        outs_e = [ce.new_coarse() for _ in range(10)]
        outs_g = [cg.new_coarse() for _ in range(10)]
        for rnd in range(2):
            for i in range(10):
                E.efpi_macro_step(ce.ctx, a, outs_e[i], [100 * rnd + i])
                E.efpi_macro_step_graph(cg.ctx, a, outs_g[i], [100 * rnd + i])
            side.synchronize()
            for i in range(10):
                assert torch.equal(outs_e[i], outs_g[i]), (rnd, i)
