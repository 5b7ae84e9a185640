"""Parity at the full size of the expanding-slab workload (Sec. 4.2 with a uniform
slab): 16384 cells, absorbing walls, the central quarter holding 4096 ions per
cell (16,777,216 ions), T_i/T_e = 0.01, l = 4 (1024 coarse blocks), at bench.py's
particle tile (4096, one workgroup per tile).  The ions are a seeded random
cell-sorted state over the slab cells (Maxwellian velocities, weight h / 4096),
given to both sides.  Bars: charge bit-exact before and after one step; one
step sampled particle by particle within 1e-5 (the oracle's start field from
its exact fixed-point charge and Newton to 1e-13); the
plain restriction within 1e-7 (eq. 4.2) on a window of blocks whose ions the
oracle restricts, and the total mass exact to rounding.
"""
import numpy as np
import pytest

import synth
from oracle import efpi as oefpi
from oracle import metrics
from oracle import pic as opic
from helpers import lib, oracle_grid, oracle_scheme, set_particles, particles_np, grid_np, x_of, relmax

pytestmark = pytest.mark.gpu

N, PPC = 16384, 4096
LO, HI = 3 * N // 8, 5 * N // 8          # the slab's cells


@pytest.fixture(scope="module")
def slab():
    E = lib()
    n_ions = (HI - LO) * PPC
    spec = E.ReplicaSpec(N, float(N), bc=E.BC_WALLS, ppc=PPC, haar_levels=4, burst_steps=20,
                         macro_dt=20.0, dt=0.1, vth=0.1, capacity=n_ions)
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=3, newton_iters_start=6, tile=4096))
    c, f, v, w = synth.random_particles(n_ions, HI - LO, seed=2016, vth=0.1, w_mean=1.0 / PPC)
    parts = ((c + LO).astype(np.int16), f, v, w)
    return dict(E=E, spec=spec, ctx=ctx, g=oracle_grid(spec), sch=oracle_scheme(spec),
                parts=parts)


def test_slab_deposit_bitexact(slab):
    E, ctx, g, parts = slab["E"], slab["ctx"], slab["g"], slab["parts"]
    set_particles(ctx, 0, *parts)
    E.efpi_deposit(ctx.ctx)
    q, _, _ = grid_np(ctx)
    assert np.array_equal(q, opic.deposit_fx(*parts[:2], parts[3], g))


def test_slab_one_step_sampled(slab):
    E, ctx, g, parts = slab["E"], slab["ctx"], slab["g"], slab["parts"]
    cell, frac, v, w = parts
    set_particles(ctx, 0, *parts)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 80, cold=True)
    E.efpi_pic_burst(ctx.ctx, 1, False)
    gc, gf, gv, gw = particles_np(ctx)
    q, _, e = grid_np(ctx)
    x0 = x_of(cell, frac, g.h)
    # the oracle's field of the start, from its exact fixed-point charge
    rho0 = opic.fx_to_density(opic.deposit_fx(cell, frac, w, g), g)
    phi0, _, ok = opic.newton_poisson(rho0, g, tol=1e-13, max_iter=200)
    assert ok
    e0 = opic.field(phi0, g)
    rng = np.random.default_rng(2)
    # random ions and the slab's two edge cells, where the field is strongest
    edge = np.nonzero((cell == LO) | (cell == HI - 1))[0]
    idx = np.concatenate([rng.choice(x0.size, 40000, replace=False),
                          rng.choice(edge, 4000, replace=False)])
    vh = v[idx].astype(np.float64) + 0.5 * g.dt * opic.gather(e0, x0[idx], g)
    x1 = x0[idx] + g.dt * vh
    assert np.all(gc[idx] >= 0)
    assert relmax(gv[idx], vh) < 1e-5
    assert np.max(np.abs(x_of(gc[idx], gf[idx], g.h) - x1)) < 1e-5 * g.h
    # the fused deposit of the pushed ions
    assert np.array_equal(q, opic.deposit_fx(gc, gf, gw, g))


def test_slab_restriction_window(slab):
    E, ctx, g, sch, parts = slab["E"], slab["ctx"], slab["g"], slab["sch"], slab["parts"]
    cell, frac, v, w = parts
    set_particles(ctx, 0, *parts)
    c = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c)
    got = c.view(2, -1).cpu().numpy()
    # blocks 400 .. 415 take the ions of cells 6399 .. 6655 only (tau = 0)
    b0, b1 = 400, 416
    sel = (cell >= 16 * b0 - 1) & (cell < 16 * b1)
    x = x_of(cell[sel], frac[sel], g.h)
    ref = oefpi.restrict_state(x, v[sel].astype(np.float64), w[sel].astype(np.float64),
                               np.ones(x.size, bool), g, sch)
    assert metrics.rel_l2(got[0, b0:b1], ref[0, b0:b1]) < 1e-7
    assert metrics.rel_l2(got[1, b0:b1], ref[1, b0:b1]) < 1e-6   # near-cancelling momentum
    total = np.sum(w.astype(np.float64)) / g.h * 2.0 ** (-sch.levels / 2.0)
    assert abs(np.sum(got[0]) / total - 1.0) < 1e-9
