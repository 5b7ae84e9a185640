"""Plain PIC over 1000 steps on the smallest workload (the fine solver of
Sec. 2.2): the ion-acoustic wave (eq. 4.1) on L = 128 with 128 cells and 200
ions per cell (25,600 ions), T_i/T_e = 0.1, Boltzmann electrons (Newton, three
iterations per step), dt = 0.1, the oracle's quiet start given to both sides,
a cell sort every 200 steps.  Bars: after every step the total fixed-point
charge equals the ions' sum of rint(w 2^40) (periodic, so no ion leaves); every
100 steps the deposit bit-exact against the oracle's deposit of the GPU's
state; after 1000 steps the energy W (the oracle's definition) within 5e-3 of
the initial kinetic energy of W_0 (the oracle's own run drifts 2.4e-3), and the
coarse density within eps = 5e-3 (eq. 4.2) of the oracle's 1000-step run.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import efpi as oefpi
from oracle import metrics
from oracle import pic as opic
from helpers import lib, oracle_grid, oracle_scheme, set_particles, particles_np, grid_np, x_of

pytestmark = pytest.mark.gpu

N, PPC, STEPS = 128, 200, 1000


def test_cfg1_thousand_steps():
    E = lib()
    spec = E.ReplicaSpec(N, float(N), ppc=PPC, haar_levels=3, dt=0.1, vth=math.sqrt(0.1))
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=3, newton_iters_start=8, tile=1024,
                                 flags=E.FLAG_SORT_BUFFER))
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    n0, u0 = synth.iaw_profile(N, float(N))
    c, f, v, w = oefpi.load_particles(n0, u0, g, sch, synth.lift_shift(2016))
    parts = (c.astype(np.int16), f.astype(np.float32), v.astype(np.float32), w.astype(np.float32))
    set_particles(ctx, 0, *parts)
    qtot = int(np.sum(np.rint(parts[3].astype(np.float64) * 2.0 ** 40).astype(np.int64)))
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 60, cold=True)
    for step in range(1, STEPS + 1):
        E.efpi_pic_burst(ctx.ctx, 1, False)
        q, _, _ = grid_np(ctx)
        assert int(q.sum()) == qtot, step
        if step % 100 == 0:
            gc, gf, _, gw = particles_np(ctx)
            assert np.array_equal(q, opic.deposit_fx(gc, gf, gw, g)), step
        if step % 200 == 0 and step < STEPS:
            E.efpi_sort(ctx.ctx)
    bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
    assert bits & (E.DEV_NAN | E.DEV_NEWTON) == 0
    # energy: time-centred velocities from the stored field
    gc, gf, gv, gw = particles_np(ctx)
    _, phi, e = grid_np(ctx)
    x = x_of(gc, gf, g.h)
    alive = gc >= 0
    vi = gv.astype(np.float64) + 0.5 * g.dt * opic.gather(e.astype(np.float64), x, g)
    x0 = x_of(*parts[:2], g.h)
    _, phi0, _ = opic.field_from_particles(x0, parts[3].astype(np.float64), np.ones(x0.size, bool), g)
    w64, v64 = parts[3].astype(np.float64), parts[2].astype(np.float64)
    W0 = opic.energy(x0, v64, w64, np.ones(x0.size, bool), phi0, g)
    W1 = opic.energy(x, vi, gw.astype(np.float64), alive, phi, g)
    kin0 = 0.5 * np.sum(w64 * v64 ** 2)
    assert abs(W1 - W0) / kin0 < 5e-3
    # the oracle's own 1000 steps from the same start
    xs, vh, al, phio = opic.pic_run(x0, v64, w64, g, STEPS)
    vio = vh + 0.5 * g.dt * opic.gather(opic.field(phio, g), xs, g)
    ref = oefpi.restrict_state(xs, vio, w64, al, g, sch)
    got = oefpi.restrict_state(x, vi, gw.astype(np.float64), alive, g, sch)
    assert metrics.rel_l2(got[0], ref[0]) < 5e-3
