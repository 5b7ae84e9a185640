"""Kinetic-electron parity at the benchmark's full size and launch configuration.

Workload: the ion-acoustic wave (eq. 4.1) on 4096 cells with 1000 ions and 1000
electrons per cell (4,096,000 of each), m_i / m_e = 1836, dt = 0.25 / omega_pe,
tile 2048 as in the full-PIC runs of bench.py.  The oracle loads the ions (quiet
start of App. C) and the Boltzmann electrons for them (eqs. 3.15-3.16); the GPU
receives the same FP32 state.  Bars: net charge bit-exact; phi within 1e-9 of
max |phi| and E within 1e-6; one two-species step sampled particle by particle
within 1e-5; the GPU's own Boltzmann electrons for the same ions bit-exact in
cells and offsets and within 1e-6 in velocities and weights (the GPU loads its
ions from the same profile, equal to the oracle's to 1e-6); total momentum and
charge conserved over a 200-step burst.
"""
import math

import numpy as np
import pytest
import torch

import synth
from oracle import efpi as oefpi
from oracle import kinetic as okin
from oracle import pic as opic
from helpers import lib, oracle_grid, to_dev, set_particles, particles_np, grid_np, x_of, \
    periodic_dx, relmax

pytestmark = pytest.mark.gpu

N, PPC = 4096, 1000
MU = 1836.0


def electrons_np(ctx):
    c, f, v, w = ctx.electrons(0)
    return (c.cpu().numpy(), f.cpu().numpy(), v.cpu().numpy(), w.cpu().numpy())


@pytest.fixture(scope="module")
def full():
    E = lib()
    spec = E.ReplicaSpec(N, float(N), ppc=PPC, haar_levels=4, burst_steps=60, macro_dt=7.5,
                         dt=0.25 / math.sqrt(MU), vth=math.sqrt(0.1),
                         closure=E.CLOSURE_KINETIC, qm_e=-MU, vth_e=math.sqrt(MU), ppc_e=PPC)
    ctx = E.Context(E.ConfigSpec([spec], newton_iters=2, newton_iters_start=8, tile=2048,
                                 flags=E.FLAG_SORT_BUFFER))
    g = oracle_grid(spec)
    sch = oefpi.Scheme(levels=4, burst_steps=60, macro_dt=7.5, ppc=PPC, vth=spec.vth)
    el = okin.Electrons(mu=MU, vth=math.sqrt(MU), ppc=PPC)
    n, u = synth.iaw_profile(N, float(N))
    c, f, v, w = oefpi.load_particles(n, u, g, sch, synth.lift_shift(2016))
    ions = (c.astype(np.int16), f.astype(np.float32), v.astype(np.float32), w.astype(np.float32))
    xi = x_of(ions[0], ions[1], g.h)
    ce, fe, ve, we, phi_b = okin.boltzmann_electrons(xi, ions[3].astype(np.float64), u, g, el,
                                                     okin.electron_shift(55))
    elec = (ce.astype(np.int16), fe.astype(np.float32), ve.astype(np.float32),
            we.astype(np.float32))
    return dict(E=E, spec=spec, ctx=ctx, g=g, el=el, ions=ions, elec=elec, u=u,
                ref_elec=(ce, fe, ve, we))


def _load(full):
    E, ctx = full["E"], full["ctx"]
    set_particles(ctx, 0, *full["ions"])
    E.efpi_set_electrons(ctx.ctx, 0, *[to_dev(a, t) for a, t in zip(
        full["elec"], (torch.int16, torch.float32, torch.float32, torch.float32))])


def test_fullsize_net_charge_and_field(full):
    E, ctx, g = full["E"], full["ctx"], full["g"]
    _load(full)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 1)
    q, phi, e = grid_np(ctx)
    ions, elec = full["ions"], full["elec"]
    ref_q = okin.net_charge_fx((ions[0], ions[1], ions[3]), (elec[0], elec[1], elec[3]), g)
    assert np.array_equal(q, ref_q)
    ref_phi = opic.linear_poisson(opic.fx_to_density(ref_q, g), g)
    assert np.max(np.abs(phi - ref_phi)) <= 1e-9 * np.max(np.abs(ref_phi))
    assert relmax(e, opic.field(ref_phi, g)) < 1e-6


def test_fullsize_two_species_step_sampled(full):
    E, ctx, g, el = full["E"], full["ctx"], full["g"], full["el"]
    _load(full)
    E.efpi_pic_burst(ctx.ctx, 1, False)
    ions, elec = full["ions"], full["elec"]
    xi0 = x_of(ions[0], ions[1], g.h)
    xe0 = x_of(elec[0], elec[1], g.h)
    ai = np.ones(xi0.size, bool)
    ae = np.ones(xe0.size, bool)
    _, _, e0 = okin.kinetic_field(xi0, ions[3].astype(np.float64), ai, xe0,
                                  elec[3].astype(np.float64), ae, g)
    rng = np.random.default_rng(3)
    for parts, x0, qm, got in ((ions, xi0, 1.0, particles_np(ctx)),
                               (elec, xe0, el.qm, electrons_np(ctx))):
        idx = rng.choice(x0.size, 20000, replace=False)
        vh = parts[2][idx].astype(np.float64) + qm * 0.5 * g.dt * opic.gather(e0, x0[idx], g)
        x1 = np.mod(x0[idx] + g.dt * vh, g.length)
        assert relmax(got[2][idx], vh) < 1e-5
        assert np.max(np.abs(periodic_dx(x_of(got[0][idx], got[1][idx], g.h), x1, g.length))) \
            < 1e-5 * g.h


def test_fullsize_boltzmann_electrons(full):
    E, ctx, g = full["E"], full["ctx"], full["g"]
    set_particles(ctx, 0, *full["ions"])
    n, u = synth.iaw_profile(N, float(N))
    # the ions' loading profile is what efpi_boltzmann_electrons takes as their velocity
    E.efpi_load_profile(ctx.ctx, 0, to_dev(n, torch.float64), to_dev(u, torch.float64), 2016)
    E.efpi_boltzmann_electrons(ctx.ctx, [55])
    E.efpi_sync(ctx.ctx)
    gi = particles_np(ctx)
    assert np.array_equal(gi[0], full["ions"][0]) and np.array_equal(gi[1], full["ions"][1])
    assert relmax(gi[3], full["ions"][3]) < 1e-6   # the oracle's ions, to the FP32 load
    c, f, v, w = electrons_np(ctx)
    rc, rf, rv, rw = full["ref_elec"]
    assert np.array_equal(c, rc) and np.array_equal(f.astype(np.float64), rf)
    assert relmax(v, rv) < 1e-6 and relmax(w, rw) < 1e-6


def test_fullsize_burst_conserves_momentum_and_charge(full):
    E, ctx = full["E"], full["ctx"]
    _load(full)
    E.efpi_pic_burst(ctx.ctx, 1, False)

    def state():
        _, _, vi, wi = particles_np(ctx)
        _, _, ve, we = electrons_np(ctx)
        q, _, _ = grid_np(ctx)
        p = np.sum(wi.astype(np.float64) * vi) + np.sum(we.astype(np.float64) * ve) / MU
        s = np.sum(np.abs(wi.astype(np.float64) * vi)) + np.sum(np.abs(we.astype(np.float64) * ve)) / MU
        return p, s, int(q.sum())

    p0, s0, q0 = state()
    E.efpi_pic_burst(ctx.ctx, 100, False)
    E.efpi_sort(ctx.ctx)
    E.efpi_pic_burst(ctx.ctx, 99, False)
    p1, _, q1 = state()
    E.efpi_sync(ctx.ctx)
    assert q1 == q0
    assert abs(p1 - p0) < 1e-5 * s0
