"""Kinetic electrons on the GPU (through the C ABI) against the oracle.

Bars: net fixed-point charge of both species bit-exact; linear Poisson phi
within 1e-9 of the FP64 oracle relative to max |phi| (two exact FP64 solvers:
prefix sums against a sparse direct solve) and the FP32 field within 1e-6;
one two-species step within 1e-5 relative (FP32 particles against FP64); loaded
electrons: cells and offsets bit-exact, velocities and weights within 1e-6;
total momentum conserved to FP32 rounding; the kinetic macro step within
eps = 1e-4 (eq. 4.2) of the oracle's, the density's perturbation about its mean
included; graph replays bit-equal to eager steps.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import efpi as oefpi
from oracle import kinetic as okin
from oracle import metrics
from oracle import pic as opic
from helpers import (lib, oracle_grid, oracle_scheme, to_dev, set_particles, particles_np,
                     grid_np, x_of, periodic_dx, relmax)

pytestmark = pytest.mark.gpu

MU = 100.0                    # m_i / m_e of the small test plasmas
VTH_E = 10.0                  # sqrt(mu): T_e = 1
DT = 0.025                    # 0.25 / omega_pe


def kspec(E, n_cells, ppc, ppc_e, **kw):
    kw.setdefault("dt", DT)
    kw.setdefault("haar_levels", 3)
    return E.ReplicaSpec(n_cells, float(n_cells), ppc=ppc, closure=E.CLOSURE_KINETIC,
                         qm_e=-MU, vth_e=VTH_E, ppc_e=ppc_e, **kw)


def make_ctx(specs, **kw):
    E = lib()
    kw.setdefault("newton_iters_start", 12)
    return E.Context(E.ConfigSpec(list(specs), **kw))


def set_electrons(ctx, replica, cell, frac, v, w):
    E = lib()
    E.efpi_set_electrons(ctx.ctx, replica, to_dev(cell, torch.int16), to_dev(frac, torch.float32),
                         to_dev(v, torch.float32), to_dev(w, torch.float32))


def electrons_np(ctx, replica=0):
    c, f, v, w = ctx.electrons(replica)
    return (c.cpu().numpy(), f.cpu().numpy(), v.cpu().numpy(), w.cpu().numpy())


def el_params(ppc_e):
    return okin.Electrons(mu=MU, vth=VTH_E, ppc=ppc_e)


def random_pair(n_cells, ppc, seed):
    ions = synth.random_particles(n_cells * ppc, n_cells, seed, vth=0.3, w_mean=1.0 / ppc)
    elec = synth.random_particles(n_cells * ppc, n_cells, seed + 1, vth=VTH_E, w_mean=1.0 / ppc,
                                  sort=False)
    return ions, elec


# ------------------------------------------------------------ deposit, field --

@pytest.mark.parametrize("n_cells,ppc", [(8, 40), (256, 30), (1024, 9), (4096, 5), (8192, 3)])
def test_net_charge_and_poisson_match_oracle(n_cells, ppc):
    E = lib()
    spec = kspec(E, n_cells, ppc, ppc, haar_levels=2)
    ctx = make_ctx([spec])
    ions, elec = random_pair(n_cells, ppc, n_cells + 3)
    set_particles(ctx, 0, *ions)
    set_electrons(ctx, 0, *elec)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 1)
    E.efpi_sync(ctx.ctx)
    q, phi, e = grid_np(ctx)
    g = oracle_grid(spec)
    ref_q = okin.net_charge_fx((ions[0], ions[1], ions[3]), (elec[0], elec[1], elec[3]), g)
    assert np.array_equal(q, ref_q)
    ref_phi = opic.linear_poisson(opic.fx_to_density(ref_q, g), g)
    assert np.max(np.abs(phi - ref_phi)) <= 1e-9 * np.max(np.abs(ref_phi))
    assert relmax(e, opic.field(ref_phi, g)) < 1e-6


def test_poisson_matches_spectral_solution():
    # The periodic second difference is diagonal in the discrete Fourier basis:
    # phi_m = rho_m h^2 / (4 sin^2(pi m / N)) for m != 0 and phi_0 = 0 (zero mean).
    E = lib()
    n, ppc = 2048, 6
    spec = kspec(E, n, ppc, ppc, haar_levels=2)
    ctx = make_ctx([spec])
    ions, elec = random_pair(n, ppc, 91)
    set_particles(ctx, 0, *ions)
    set_electrons(ctx, 0, *elec)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 1)
    q, phi, _ = grid_np(ctx)
    h = spec.length / n
    rho_m = np.fft.fft(q.astype(np.float64) / 2.0 ** 40 / h)
    m = np.arange(n)
    lam = 4.0 * np.sin(np.pi * m / n) ** 2 / h ** 2
    lam[0] = 1.0
    phi_m = rho_m / lam
    phi_m[0] = 0.0
    want = np.fft.ifft(phi_m).real
    assert np.max(np.abs(phi - want)) <= 1e-9 * np.max(np.abs(want))


# ------------------------------------------------------------------ stepping --

@pytest.mark.parametrize("n_cells,ppc,steps", [(256, 40, 1), (1024, 12, 1), (512, 20, 4)])
def test_two_species_steps_match_oracle(n_cells, ppc, steps):
    E = lib()
    spec = kspec(E, n_cells, ppc, ppc)
    ctx = make_ctx([spec])
    ions, elec = random_pair(n_cells, ppc, 50 + n_cells)
    set_particles(ctx, 0, *ions)
    set_electrons(ctx, 0, *elec)
    E.efpi_pic_burst(ctx.ctx, steps, False)
    E.efpi_sync(ctx.ctx)
    g = oracle_grid(spec)
    el = el_params(ppc)
    xi0 = x_of(ions[0], ions[1], g.h)
    xe0 = x_of(elec[0], elec[1], g.h)
    (xi, vi), (xe, ve), phi = okin.kinetic_run(
        (xi0, ions[2].astype(np.float64), ions[3].astype(np.float64)),
        (xe0, elec[2].astype(np.float64), elec[3].astype(np.float64)), g, el, steps)
    tol = 1e-5 if steps == 1 else 1e-4
    gc, gf, gv, gw = particles_np(ctx)
    assert relmax(gv, vi) < tol
    assert np.max(np.abs(periodic_dx(x_of(gc, gf, g.h), xi, g.length))) < tol * g.h
    ec, ef, ev, ew = electrons_np(ctx)
    assert relmax(ev, ve) < tol
    assert np.max(np.abs(periodic_dx(x_of(ec, ef, g.h), xe, g.length))) < tol * g.h * 10
    assert np.array_equal(ew, elec[3])
    q, gphi, ge = grid_np(ctx)
    assert np.array_equal(q, okin.net_charge_fx((gc, gf, gw), (ec, ef, ew), g))
    assert relmax(ge, opic.field(phi, g)) < tol * 10


def test_momentum_and_charge_conserved_over_a_burst():
    E = lib()
    n, ppc = 512, 40
    spec = kspec(E, n, ppc, ppc)
    ctx = make_ctx([spec])
    ions, elec = random_pair(n, ppc, 7)
    set_particles(ctx, 0, *ions)
    set_electrons(ctx, 0, *elec)
    E.efpi_pic_burst(ctx.ctx, 1, False)

    def state():
        _, _, vi, wi = particles_np(ctx)
        _, _, ve, we = electrons_np(ctx)
        q, _, _ = grid_np(ctx)
        p = np.sum(wi.astype(np.float64) * vi) + np.sum(we.astype(np.float64) * ve) / MU
        s = np.sum(np.abs(wi.astype(np.float64) * vi)) + np.sum(np.abs(we * ve)) / MU
        return p, s, int(q.sum())

    p0, s0, q0 = state()
    E.efpi_pic_burst(ctx.ctx, 60, False)
    p1, _, q1 = state()
    assert q1 == q0
    assert abs(p1 - p0) < 2e-5 * s0


# ------------------------------------------------------------------- loading --

def test_load_electrons_matches_oracle():
    E = lib()
    n, ppc_e = 512, 37
    spec = kspec(E, n, 20, ppc_e)
    ctx = make_ctx([spec])
    dens, u = synth.iaw_profile(n, float(n))
    E.efpi_load_profile(ctx.ctx, 0, to_dev(dens, torch.float64), to_dev(u, torch.float64), 5)
    ne = np.exp(0.3 * np.sin(2 * np.pi * np.arange(n) / n))
    E.efpi_load_electrons(ctx.ctx, 0, to_dev(ne, torch.float64), to_dev(u, torch.float64), 99)
    c, f, v, w = electrons_np(ctx)
    rc, rf, rv, rw = okin.load_electrons(ne, u, oracle_grid(spec), el_params(ppc_e), 99)
    assert np.array_equal(c, rc) and np.array_equal(f.astype(np.float64), rf)
    assert relmax(v, rv) < 1e-6 and relmax(w, rw) < 1e-6


def test_boltzmann_electrons_match_oracle():
    E = lib()
    n, ppc, ppc_e = 256, 64, 48
    spec = kspec(E, n, ppc, ppc_e)
    ctx = make_ctx([spec])
    dens, u = synth.iaw_profile(n, float(n))
    E.efpi_load_profile(ctx.ctx, 0, to_dev(dens, torch.float64), to_dev(u, torch.float64), 17)
    E.efpi_boltzmann_electrons(ctx.ctx, [1234])
    E.efpi_sync(ctx.ctx)
    ci, fi, vi, wi = particles_np(ctx)
    c, f, v, w = electrons_np(ctx)
    g = oracle_grid(spec)
    rc, rf, rv, rw, _ = okin.boltzmann_electrons(x_of(ci, fi, g.h), wi.astype(np.float64), u, g,
                                                 el_params(ppc_e), okin.electron_shift(1234))
    assert np.array_equal(c, rc) and np.array_equal(f.astype(np.float64), rf)
    assert relmax(v, rv) < 1e-6 and relmax(w, rw) < 1e-6
    # global neutrality of the equilibrium
    assert np.sum(w.astype(np.float64)) == pytest.approx(np.sum(wi.astype(np.float64)), rel=2e-6)


def test_electron_calls_check_state():
    E = lib()
    plain = make_ctx([E.ReplicaSpec(64, 64.0, ppc=4)])
    z = torch.zeros(64, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EfpiError):
        E.efpi_load_electrons(plain.ctx, 0, z, z, 1)
    with pytest.raises(E.EfpiError):
        E.efpi_boltzmann_electrons(plain.ctx, [1])
    spec = kspec(E, 64, 4, 4, haar_levels=2)
    ctx = make_ctx([spec])
    ones = torch.ones(64, dtype=torch.float64, device="cuda")
    E.efpi_load_profile(ctx.ctx, 0, ones, z, 3)
    E.efpi_load_electrons(ctx.ctx, 0, ones, z, 4)
    E.efpi_pic_burst(ctx.ctx, 2, False)
    with pytest.raises(E.EfpiError):      # ions at a half step: their lift profile is stale
        E.efpi_boltzmann_electrons(ctx.ctx, [5])
    with pytest.raises(E.EfpiError):
        E.efpi_reset_electrons(plain.ctx, [5])
    E.efpi_load_electrons(ctx.ctx, 0, ones, z, 5)   # electrons may be replaced at any time
    E.efpi_sync(ctx.ctx)


# ---------------------------------------------------------------- macro step --

def _kinetic_start(E, spec, seed):
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    n, u = synth.iaw_profile(spec.n_cells, spec.length, 0.2, n_nodes=g.n_nodes)
    c, f, v, w = oefpi.load_particles(n, u, g, sch, synth.lift_shift(seed))
    x = x_of(c, f, g.h)
    return oefpi.restrict_state(x, v.astype(np.float32).astype(np.float64),
                                w.astype(np.float32).astype(np.float64), np.ones(x.size, bool),
                                g, sch)


def test_kinetic_macro_step_matches_oracle():
    E = lib()
    spec = kspec(E, 256, 64, 64, burst_steps=20, macro_dt=2.0, vth=0.316)
    ctx = make_ctx([spec])
    c0 = _kinetic_start(E, spec, 61)
    shift = synth.lift_shift(62)
    cin = to_dev(c0.ravel(), torch.float64)
    cout = ctx.new_coarse()
    E.efpi_macro_step(ctx.ctx, cin, cout, [shift])
    E.efpi_sync(ctx.ctx)
    ref, _ = okin.kinetic_macro_step(c0, oracle_grid(spec), oracle_scheme(spec), el_params(64),
                                     shift)
    got = cout.view(2, -1).cpu().numpy()
    for m in range(2):
        assert metrics.rel_l2(got[m], ref[m]) < 1e-4
    # the wave itself: the density perturbation about its mean
    pert = metrics.rel_l2(got[0] - got[0].mean(), ref[0] - ref[0].mean())
    assert pert < 1e-4


def test_kinetic_graph_replays_equal_eager():
    E = lib()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        spec = kspec(E, 256, 32, 32, burst_steps=10, macro_dt=1.0, vth=0.316)
        ce, cg = make_ctx([spec]), make_ctx([spec])
        c0 = to_dev(_kinetic_start(E, spec, 71).ravel(), torch.float64)
        ae, ag = c0.clone(), c0.clone()
        be, bg = ce.new_coarse(), cg.new_coarse()
        for i in range(4):
            sh = [synth.lift_shift(80 + i)]
            E.efpi_macro_step(ce.ctx, ae, be, sh)
            E.efpi_macro_step_graph(cg.ctx, ag, bg, sh)
            side.synchronize()
            assert torch.equal(be, bg), f"step {i}"
            ae, be = be, ae
            ag, bg = bg, ag
        assert E.efpi_sync(cg.ctx, raise_on_error=False) == E.efpi_sync(ce.ctx, raise_on_error=False)


def test_two_replica_context_equals_single_contexts():
    """Replicas of different sizes in one kinetic context (shared launches) give
    the same bits as each replica alone."""
    E = lib()
    specs = [kspec(E, 256, 32, 24, burst_steps=10, macro_dt=1.0, vth=0.316),
             kspec(E, 512, 20, 16, burst_steps=10, macro_dt=1.0, vth=0.316)]
    both = make_ctx(specs)
    starts = [_kinetic_start(E, s, 100 + i) for i, s in enumerate(specs)]
    cin = to_dev(np.concatenate([c.ravel() for c in starts]), torch.float64)
    out = both.new_coarse()
    shifts = [synth.lift_shift(110), synth.lift_shift(111)]
    E.efpi_macro_step(both.ctx, cin, out, shifts)
    E.efpi_sync(both.ctx, raise_on_error=False)
    for r, s in enumerate(specs):
        one = make_ctx([s])
        o1 = one.new_coarse()
        E.efpi_macro_step(one.ctx, to_dev(starts[r].ravel(), torch.float64), o1, [shifts[r]])
        E.efpi_sync(one.ctx, raise_on_error=False)
        assert torch.equal(both.split_coarse(out)[r].reshape(-1), o1), f"replica {r}"


def test_sort_orders_electrons_and_keeps_the_dynamics():
    E = lib()
    n, ppc = 256, 24
    spec = kspec(E, n, ppc, ppc, haar_levels=2)
    ctxs = [make_ctx([spec], flags=E.FLAG_SORT_BUFFER) for _ in range(2)]
    ions, elec = random_pair(n, ppc, 33)
    for c in ctxs:
        set_particles(c, 0, *ions)
        set_electrons(c, 0, *elec)
        E.efpi_pic_burst(c.ctx, 30, False)
    before = electrons_np(ctxs[0])
    E.efpi_sort(ctxs[0].ctx)
    after = electrons_np(ctxs[0])
    assert np.all(np.diff(after[0].astype(np.int64)) >= 0)
    key = lambda s: np.lexsort((s[3], s[2], s[1], s[0]))
    for a, b in zip((x[key(before)] for x in before), (x[key(after)] for x in after)):
        assert np.array_equal(a, b)
    for c in ctxs:
        E.efpi_pic_burst(c.ctx, 5, False)
    qa, pa, _ = grid_np(ctxs[0])
    qb, pb, _ = grid_np(ctxs[1])
    assert np.array_equal(qa, qb)
    for c in ctxs:
        E.efpi_sync(c.ctx)


def test_reset_electrons_matches_oracle_and_restarts_the_leapfrog():
    """Reset in the middle of a run (the control run of Sec. 4.1): the electrons
    equal the oracle's reset of the GPU's current ions, the ions are untouched,
    and the next step kicks the electrons by half a step and the ions by a full one."""
    E = lib()
    n, ppc, ppc_e = 256, 48, 40
    spec = kspec(E, n, ppc, ppc_e)
    ctx = make_ctx([spec])
    dens, u = synth.iaw_profile(n, float(n))
    E.efpi_load_profile(ctx.ctx, 0, to_dev(dens, torch.float64), to_dev(u, torch.float64), 3)
    E.efpi_boltzmann_electrons(ctx.ctx, [4])
    E.efpi_pic_burst(ctx.ctx, 7, False)
    ions = particles_np(ctx)
    _, _, e_now = grid_np(ctx)
    E.efpi_reset_electrons(ctx.ctx, [77])
    E.efpi_sync(ctx.ctx)
    g = oracle_grid(spec)
    ci, fi, vi, wi = ions
    xi = x_of(ci, fi, g.h)
    vc = vi.astype(np.float64) + 0.5 * g.dt * opic.gather(e_now.astype(np.float64), xi, g)
    rc, rf, rv, rw, _ = okin.reset_electrons(xi, vc, wi.astype(np.float64), g, el_params(ppc_e),
                                             okin.electron_shift(77))
    c, f, v, w = electrons_np(ctx)
    assert np.array_equal(c, rc) and np.array_equal(f.astype(np.float64), rf)
    assert relmax(v, rv) < 1e-6 and relmax(w, rw) < 1e-6
    after = particles_np(ctx)
    for a, b in zip(ions, after):
        assert np.array_equal(a, b)
    # one more step: field of both species at the current positions, ions a full
    # kick from their half-step velocities, electrons a half kick from integer time
    E.efpi_pic_burst(ctx.ctx, 1, False)
    xe = x_of(c, f, g.h)
    al_i = np.ones(xi.size, bool)
    al_e = np.ones(xe.size, bool)
    _, _, e0 = okin.kinetic_field(xi, wi.astype(np.float64), al_i, xe, w.astype(np.float64),
                                  al_e, g)
    xi1, vi1, _ = okin.species_step(xi, vi.astype(np.float64), al_i, 1.0, e0, g)
    xe1, ve1, _ = okin.species_step(xe, v.astype(np.float64), al_e, -MU / 2.0, e0, g)
    gc, gf, gv, _ = particles_np(ctx)
    assert relmax(gv, vi1) < 1e-5
    ec, ef, ev, _ = electrons_np(ctx)
    assert relmax(ev, ve1) < 1e-5
    assert np.max(np.abs(periodic_dx(x_of(ec, ef, g.h), xe1, g.length))) < 1e-4
    E.efpi_sync(ctx.ctx)


def test_timing_counts_ion_and_electron_launches():
    E = lib()
    spec = kspec(E, 256, 16, 16, haar_levels=2)
    ctx = make_ctx([spec])
    ions, elec = random_pair(256, 16, 12)
    set_particles(ctx, 0, *ions)
    set_electrons(ctx, 0, *elec)
    E.efpi_timing(ctx.ctx, True)
    E.efpi_pic_burst(ctx.ctx, 5, False)
    ms_e, n_e = E.efpi_timing_read_electrons(ctx.ctx)
    ms_i, n_i = E.efpi_timing_read(ctx.ctx)
    E.efpi_timing(ctx.ctx, False)
    assert n_e == 5 and n_i == 5 and ms_e > 0.0 and ms_i > 0.0
    plain = make_ctx([E.ReplicaSpec(64, 64.0, ppc=4)])
    with pytest.raises(E.EfpiError):
        E.efpi_timing_read_electrons(plain.ctx)
    E.efpi_sync(ctx.ctx)
