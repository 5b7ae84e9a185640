"""GPU path (through the C ABI) against the CPU oracle on the same seeded inputs.

Bars: fixed-point grid charge bit-exact; potential within 1e-10 absolute and
field within 1e-6 relative after converged Newton (FP64 on both sides, the
field rounded to FP32 on the GPU); one fine step of FP32 particles and field
within 1e-5 relative of the FP64 oracle; lifted particles: cells and offsets
bit-exact, velocities and weights within 1e-6 relative; burst-averaged coarse
coefficients and the projected state within eps = 1e-4 (eq. 4.2), and so is the
density's perturbation about its mean (the wave itself: a whole-array eps of the
density 1 + 0.2 cos would hide a larger error of its amplitude).  Measured:
1e-9 to 3e-6 (FP32 against FP64 over a 20-step burst).
"""
import numpy as np
import pytest
import torch

import synth
from oracle import efpi as oefpi
from oracle import metrics
from oracle import pic as opic
from helpers import (lib, oracle_grid, oracle_scheme, to_dev, set_particles, particles_np,
                     grid_np, x_of, periodic_dx, relmax)

pytestmark = pytest.mark.gpu


def pert_eps(a, b):
    """eps of eq. 4.2 between the perturbations of two arrays about their means
    (for the density of the wave, 1 + 0.2 cos: the wave's own error)."""
    return metrics.rel_l2(a - a.mean(), b - b.mean())


def make_ctx(specs, **kw):
    E = lib()
    return E.Context(E.ConfigSpec(list(specs), **kw))


def iaw_particles(spec, seed, delta=0.2):
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    n, u = synth.iaw_profile(spec.n_cells, spec.length, delta, n_nodes=g.n_nodes)
    c, f, v, w = oefpi.load_particles(n, u, g, sch, synth.lift_shift(seed))
    return (c.astype(np.int16), f.astype(np.float32), v.astype(np.float32), w.astype(np.float32))


def slab_particles(spec, seed):
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    n, u = synth.slab_profile(spec.n_cells)
    c, f, v, w = oefpi.load_particles(n, u, g, sch, synth.lift_shift(seed))
    return (c.astype(np.int16), f.astype(np.float32), v.astype(np.float32), w.astype(np.float32))


# ------------------------------------------------------------------ deposit --

@pytest.mark.parametrize("n_cells,bc,n,srt,dead,tile", [
    (8, 0, 3000, False, 0.0, 0),
    (128, 0, 25600 + 123, True, 0.05, 1024),
    (256, 1, 30001, False, 0.1, 0),
    (4096, 0, 4096 * 50 + 77, True, 0.0, 0),
    (16384, 1, 300000, True, 0.02, 8192),
])
def test_deposit_bitexact(n_cells, bc, n, srt, dead, tile):
    E = lib()
    spec = E.ReplicaSpec(n_cells, 0.75 * n_cells, bc=bc, ppc=1, haar_levels=2, capacity=n)
    ctx = make_ctx([spec], tile=tile)
    cell, frac, v, w = synth.random_particles(n, n_cells, seed=n_cells + n, sort=srt,
                                              dead_fraction=dead)
    set_particles(ctx, 0, cell, frac, v, w)
    E.efpi_deposit(ctx.ctx)
    q, _, _ = grid_np(ctx)
    ref = opic.deposit_fx(cell, frac, w, oracle_grid(spec))
    assert np.array_equal(q, ref)
    alive = cell >= 0
    assert int(q.sum()) == int(np.rint(w[alive].astype(np.float64) * 2.0 ** 40).astype(np.int64).sum())


def test_deposit_empty_store():
    E = lib()
    spec = E.ReplicaSpec(64, 64.0, ppc=4)
    ctx = make_ctx([spec])
    z16 = torch.zeros(0, dtype=torch.int16, device="cuda")
    z32 = torch.zeros(0, dtype=torch.float32, device="cuda")
    E.efpi_set_particles(ctx.ctx, 0, z16, z32, z32, z32)
    E.efpi_deposit(ctx.ctx)
    q, _, _ = grid_np(ctx)
    assert not q.any()


# ------------------------------------------------------------------- Newton --

# Sizes cover every launch shape of the solve: fewer threads than one wave (8,
# 32), exactly one wave (64), two to eight waves (128 .. 16384), 1 to 32 rows
# per thread, both boundary conditions.
@pytest.mark.parametrize("n_cells,bc", [(8, 0), (32, 0), (64, 0), (128, 0), (1024, 0), (4096, 0),
                                        (8192, 0), (16384, 0), (32, 1), (64, 1), (128, 1),
                                        (256, 1), (2048, 1), (16384, 1)])
def test_newton_matches_oracle(n_cells, bc):
    E = lib()
    spec = E.ReplicaSpec(n_cells, float(n_cells), bc=bc, ppc=8 if n_cells > 4096 else 32,
                         haar_levels=2)
    ctx = make_ctx([spec])
    parts = iaw_particles(spec, 3) if bc == 0 else slab_particles(spec, 3)
    set_particles(ctx, 0, *parts)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 80, cold=True)
    bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
    q, phi, e = grid_np(ctx)
    g = oracle_grid(spec)
    rho = opic.fx_to_density(opic.deposit_fx(*parts[:2], parts[3], g), g)
    phi_ref, _, ok = opic.newton_poisson(rho, g, tol=1e-13, max_iter=200)
    assert ok
    assert np.max(np.abs(phi - phi_ref)) < 1e-9
    assert relmax(e, opic.field(phi_ref, g)) < 1e-6
    assert bits & E.DEV_NAN == 0


def test_newton_mixed_launch_group():
    """Replicas of 8 .. 256 cells share one launch of the solve (one row per
    thread), so the smaller ones leave lanes and whole waves idle."""
    E = lib()
    sizes = [(256, 0), (8, 0), (64, 1), (32, 0), (128, 1), (16, 1)]
    specs = [E.ReplicaSpec(n, float(n), bc=bc, ppc=24, haar_levels=2) for n, bc in sizes]
    ctx = make_ctx(specs)
    parts = []
    for r, sp in enumerate(specs):
        pr = iaw_particles(sp, 11 + r) if sp.bc == 0 else slab_particles(sp, 11 + r)
        set_particles(ctx, r, *pr)
        parts.append(pr)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 80, cold=True)
    bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
    assert bits & E.DEV_NAN == 0
    for r, sp in enumerate(specs):
        q, phi, e = grid_np(ctx, r)
        g = oracle_grid(sp)
        rho = opic.fx_to_density(opic.deposit_fx(*parts[r][:2], parts[r][3], g), g)
        phi_ref, _, ok = opic.newton_poisson(rho, g, tol=1e-13, max_iter=200)
        assert ok
        assert np.max(np.abs(phi - phi_ref)) < 1e-9, (r, sp.n_cells, sp.bc)
        assert relmax(e, opic.field(phi_ref, g)) < 1e-6, (r, sp.n_cells, sp.bc)


# ----------------------------------------------------------------- one step --

@pytest.mark.parametrize("n_cells,bc,ppc", [(256, 0, 100), (1024, 0, 33), (512, 1, 40)])
def test_one_step_matches_oracle(n_cells, bc, ppc):
    E = lib()
    spec = E.ReplicaSpec(n_cells, float(n_cells), bc=bc, ppc=ppc, haar_levels=3,
                         vth=0.3 if bc == 0 else 0.1)
    ctx = make_ctx([spec])
    parts = iaw_particles(spec, 5) if bc == 0 else slab_particles(spec, 5)
    cell, frac, v, w = parts
    set_particles(ctx, 0, *parts)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 80)
    E.efpi_pic_burst(ctx.ctx, 1, False)
    gc, gf, gv, gw = particles_np(ctx)
    q, phi, e = grid_np(ctx)
    # oracle, FP64 from the same FP32 state
    g = oracle_grid(spec)
    x0 = x_of(cell, frac, g.h)
    alive = np.ones(x0.size, bool)
    _, phi0, e0 = opic.field_from_particles(x0, w.astype(np.float64), alive, g)
    vh = v.astype(np.float64) + 0.5 * g.dt * opic.gather(e0, x0, g)
    x1 = x0 + g.dt * vh
    x1, alive = opic.apply_bc(x1, alive, g)
    _, phi1, e1 = opic.field_from_particles(x1, w.astype(np.float64), alive, g, phi0)
    # particle state
    assert np.array_equal(gc >= 0, alive)
    assert relmax(gv, vh) < 1e-5
    xg = x_of(gc, gf, g.h)
    dx = periodic_dx(xg[alive], x1[alive], g.length) if bc == 0 else xg[alive] - x1[alive]
    assert np.max(np.abs(dx)) < 1e-5 * g.h
    assert np.array_equal(gw, w)
    # field after the step
    assert relmax(e, e1) < 1e-5
    # the fused deposit of the pushed particles is bit-exact
    assert np.array_equal(q, opic.deposit_fx(gc, gf, gw, g))


# --------------------------------------------------------------------- lift --

@pytest.mark.parametrize("n_cells,bc,levels,linear,ppc", [(256, 0, 3, 1, 64), (256, 0, 2, 0, 17),
                                                          (512, 1, 4, 1, 40)])
def test_lift_matches_oracle(n_cells, bc, levels, linear, ppc):
    E = lib()
    spec = E.ReplicaSpec(n_cells, float(n_cells), bc=bc, ppc=ppc, haar_levels=levels,
                         lift_linear=linear, vth=0.25)
    ctx = make_ctx([spec])
    nc = n_cells >> levels
    coarse = synth.random_coarse(nc, seed=21, levels=levels)
    if bc == 1:
        coarse[:, : nc // 4] = 0.0
        coarse[:, -nc // 4:] = 0.0
    shift = synth.lift_shift(21)
    E.efpi_lift(ctx.ctx, to_dev(coarse.ravel(), torch.float64), [shift])
    gc, gf, gv, gw = particles_np(ctx)
    oc, of, ov, ow = oefpi.lift(coarse, oracle_grid(spec), oracle_scheme(spec), shift)
    assert gc.size == oc.size
    assert np.array_equal(gc.astype(np.int64), oc)
    assert np.array_equal(gf, of.astype(np.float32))
    assert relmax(gv, ov) < 1e-6
    assert relmax(gw, ow) < 1e-6


@pytest.mark.parametrize("bc,levels,ppc", [(0, 2, 37), (1, 3, 50), (0, 6, 11), (1, 6, 64)])
def test_lift_deposit_equals_the_deposit_pass(bc, levels, ppc):
    """The lift deposits the charge of the ions it writes (blocks of up to 64
    cells): the same int64 grid as the deposit pass over the stored ions."""
    E = lib()
    n = 1024
    spec = E.ReplicaSpec(n, float(n), bc=bc, ppc=ppc, haar_levels=levels, vth=0.316)
    ctx = make_ctx([spec])
    n0, u0 = synth.slab_profile(n) if bc else synth.iaw_profile(n, float(n))
    E.efpi_load_profile(ctx.ctx, 0, to_dev(n0, torch.float64), to_dev(u0, torch.float64), 5)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 40, cold=True)
    c0 = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c0)
    E.efpi_lift(ctx.ctx, c0, [99])
    q_lift = ctx.grid(0)[0].clone()
    E.efpi_deposit(ctx.ctx)
    q_pass = ctx.grid(0)[0].clone()
    assert int(q_lift.abs().sum().item()) > 0
    assert torch.equal(q_lift, q_pass)
    assert E.efpi_sync(ctx.ctx, raise_on_error=False) == 0


def test_load_profile_matches_oracle():
    E = lib()
    spec = E.ReplicaSpec(128, 128.0, ppc=50, haar_levels=2)
    ctx = make_ctx([spec])
    n, u = synth.iaw_profile(128, 128.0)
    shift = synth.lift_shift(4)
    E.efpi_load_profile(ctx.ctx, 0, to_dev(n, torch.float64), to_dev(u, torch.float64), shift)
    gc, gf, gv, gw = particles_np(ctx)
    oc, of, ov, ow = oefpi.load_particles(n, u, oracle_grid(spec), oracle_scheme(spec), shift)
    assert np.array_equal(gc.astype(np.int64), oc) and np.array_equal(gf, of.astype(np.float32))
    assert relmax(gv, ov) < 1e-6 and relmax(gw, ow) < 1e-6


# ---------------------------------------------------------- burst + project --

def _burst_compare(spec, parts, seed_tag, newton_iters=2):
    E = lib()
    ctx = make_ctx([spec], newton_iters=newton_iters)
    set_particles(ctx, 0, *parts)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 100, cold=True)
    E.efpi_pic_burst(ctx.ctx, spec.burst_steps, True)
    snap = ctx.new_snap()
    E.efpi_restrict(ctx.ctx, snap)
    nxt = ctx.new_coarse()
    E.efpi_project(ctx.ctx, snap, nxt)
    E.efpi_sync(ctx.ctx)
    gs = snap.view(spec.burst_steps + 1, 2, -1).cpu().numpy()
    gn = nxt.view(2, -1).cpu().numpy()
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    cell, frac, v, w = parts
    os_, *_ = oefpi.pic_burst(x_of(cell, frac, g.h), v.astype(np.float64), w.astype(np.float64),
                              g, sch)
    on = oefpi.project(os_, g.dt, sch.macro_dt)
    for m in range(2):
        assert metrics.rel_l2(gs[:, m].mean(axis=0), os_[:, m].mean(axis=0)) < 1e-4
        assert metrics.rel_l2(gn[m], on[m]) < 1e-4
    # the wave itself, not its mean: the density perturbation about its mean
    assert pert_eps(gn[0], on[0]) < 1e-4
    return gs, gn, os_, on


@pytest.mark.parametrize("coev", [1, 0])
def test_burst_restriction_periodic(coev):
    E = lib()
    spec = E.ReplicaSpec(512, 512.0, ppc=100, haar_levels=4, burst_steps=20, macro_dt=20.0,
                         coevolving=coev)
    _burst_compare(spec, iaw_particles(spec, 8), "iaw")


def test_burst_restriction_walls():
    E = lib()
    spec = E.ReplicaSpec(512, 512.0, bc=1, ppc=60, haar_levels=3, burst_steps=10, macro_dt=8.0,
                         vth=0.1)
    # the slab edge accelerates: three Newton iterations per step keep the last
    # update below the status threshold (remaining error ~1e-10)
    _burst_compare(spec, slab_particles(spec, 9), "slab", newton_iters=3)


def test_free_streaming_snapshots_equal():
    # App. B pin on the GPU: with E = 0 every co-evolving snapshot is the same.
    E = lib()
    spec = E.ReplicaSpec(256, 256.0, closure=E.CLOSURE_NOFIELD, ppc=40, haar_levels=3,
                         burst_steps=8, macro_dt=6.0)
    ctx = make_ctx([spec])
    set_particles(ctx, 0, *iaw_particles(spec, 10))
    E.efpi_pic_burst(ctx.ctx, spec.burst_steps, True)
    snap = ctx.new_snap()
    E.efpi_restrict(ctx.ctx, snap)
    s = snap.view(spec.burst_steps + 1, 2, -1).cpu().numpy()
    assert metrics.rel_l2(s, np.broadcast_to(s[0], s.shape)) < 1e-6


def test_macro_step_matches_oracle():
    E = lib()
    spec = E.ReplicaSpec(512, 512.0, ppc=100, haar_levels=4, burst_steps=20, macro_dt=20.0)
    ctx = make_ctx([spec])
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    parts = iaw_particles(spec, 11)
    x = x_of(parts[0], parts[1], g.h)
    c0 = oefpi.restrict_state(x, parts[2].astype(np.float64), parts[3].astype(np.float64),
                              np.ones(x.size, bool), g, sch)
    shift = synth.lift_shift(12)
    cin = to_dev(c0.ravel(), torch.float64)
    cout = ctx.new_coarse()
    E.efpi_macro_step(ctx.ctx, cin, cout, [shift])
    E.efpi_sync(ctx.ctx)
    ref, _, _ = oefpi.macro_step(c0, g, sch, shift)
    got = cout.view(2, -1).cpu().numpy()
    for m in range(2):
        assert metrics.rel_l2(got[m], ref[m]) < 1e-4
    assert pert_eps(got[0], ref[0]) < 1e-4
    # second call from the same input: identical bits (deterministic)
    cout2 = ctx.new_coarse()
    E.efpi_macro_step(ctx.ctx, cin, cout2, [shift])
    torch.cuda.synchronize()
    assert torch.equal(cout, cout2)


@pytest.mark.parametrize("ne", [1, 2, 4])
def test_short_burst_macro_step_matches_oracle(ne):
    """Macro steps with the short bursts the benchmark's burst-length sweep runs
    (N_e = 1, 2, 4: the LS slope of eq. 3.18 through two to five snapshots)."""
    E = lib()
    spec = E.ReplicaSpec(512, 512.0, ppc=100, haar_levels=4, burst_steps=ne, macro_dt=7.5)
    ctx = make_ctx([spec])
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    parts = iaw_particles(spec, 14)
    x = x_of(parts[0], parts[1], g.h)
    c0 = oefpi.restrict_state(x, parts[2].astype(np.float64), parts[3].astype(np.float64),
                              np.ones(x.size, bool), g, sch)
    shift = synth.lift_shift(15)
    cout = ctx.new_coarse()
    E.efpi_macro_step(ctx.ctx, to_dev(c0.ravel(), torch.float64), cout, [shift])
    assert E.efpi_sync(ctx.ctx, raise_on_error=False) == 0
    ref, _, _ = oefpi.macro_step(c0, g, sch, shift)
    got = cout.view(2, -1).cpu().numpy()
    for m in range(2):
        assert metrics.rel_l2(got[m], ref[m]) < 1e-4
    assert pert_eps(got[0], ref[0]) < 1e-4


@pytest.mark.parametrize("bc", [0, 1])
def test_macro_step_equals_composed_calls(bc):
    """efpi_macro_step (fused lift preparation, fused restriction and projection)
    gives the same bits as the single-step calls lift, burst, restrict, project,
    each path in a fresh context."""
    E = lib()
    spec = E.ReplicaSpec(512, 512.0, bc=bc, ppc=64, haar_levels=3, burst_steps=10,
                         macro_dt=6.0, vth=0.316 if bc == 0 else 0.1)
    parts = iaw_particles(spec, 21) if bc == 0 else slab_particles(spec, 21)
    first = make_ctx([spec], newton_iters=3, newton_iters_start=6)
    set_particles(first, 0, *parts)
    cin = first.new_coarse()
    E.efpi_restrict_state(first.ctx, cin)
    E.efpi_sync(first.ctx)
    shift = synth.lift_shift(22)
    a = make_ctx([spec], newton_iters=3, newton_iters_start=6)
    out_a = a.new_coarse()
    E.efpi_macro_step(a.ctx, cin, out_a, [shift])
    b = make_ctx([spec], newton_iters=3, newton_iters_start=6)
    E.efpi_lift(b.ctx, cin, [shift])
    E.efpi_pic_burst(b.ctx, spec.burst_steps, True)
    snap = b.new_snap()
    E.efpi_restrict(b.ctx, snap)
    out_b = b.new_coarse()
    E.efpi_project(b.ctx, snap, out_b)
    E.efpi_sync(a.ctx, raise_on_error=False)
    E.efpi_sync(b.ctx, raise_on_error=False)
    assert torch.equal(out_a, out_b)


# -------------------------------------------------------------- status/error --

def test_invalid_config_rejected():
    E = lib()
    with pytest.raises(E.EfpiError):
        make_ctx([E.ReplicaSpec(100, 100.0)])  # not a power of two


@pytest.mark.parametrize("n_cells,bc", [(128, 0), (2048, 1), (4096, 0), (16384, 1)])
def test_potential_round_trip(n_cells, bc):
    """The field solve stores the potential in its own order (pairs of each thread's
    nodes side by side); efpi_set_potential and efpi_get_grid translate, so a
    potential comes back bit for bit, node N of a walled grid included."""
    E = lib()
    ctx = make_ctx([E.ReplicaSpec(n_cells, float(n_cells), bc=bc, ppc=1)])
    nn = n_cells + (1 if bc == 1 else 0)
    phi = np.random.default_rng(n_cells).standard_normal(nn)
    E.efpi_set_potential(ctx.ctx, 0, to_dev(phi, torch.float64))
    _, got, _ = grid_np(ctx)
    assert np.array_equal(got[:nn], phi)


def test_newton_status_flag():
    E = lib()
    spec = E.ReplicaSpec(256, 256.0, bc=1, ppc=16, haar_levels=2, vth=0.1)
    ctx = make_ctx([spec], newton_tol=1e-30)
    set_particles(ctx, 0, *slab_particles(spec, 2))
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 1, cold=True)
    bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
    assert bits & E.DEV_NEWTON


@pytest.mark.parametrize("w_big,wv_big,flag", [(15.9, 15.9, False), (16.0, 1.0, True),
                                               (40.0, 1.0, True), (1.0, 16.0, True)])
def test_weight_bound_flag(w_big, wv_big, flag):
    """The particle pass keeps its per-lane bin sums exact for ion weights and
    snapshot momenta |w V| below 16 (integer-valued binary64 below 2^53); one ion
    at or above it sets EFPI_DEV_WEIGHT, in the deposit (w) or the restriction (w V)."""
    E = lib()
    spec = E.ReplicaSpec(64, 64.0, ppc=4, haar_levels=2)
    ctx = make_ctx([spec])
    rng = np.random.default_rng(3)
    n = 256
    cell = np.sort(rng.integers(0, 64, n)).astype(np.int16)
    frac = rng.random(n).astype(np.float32)
    v = rng.normal(0.0, 0.1, n).astype(np.float32)
    w = np.full(n, 0.25, np.float32)
    w[17] = w_big
    w[200], v[200] = 1.0, wv_big   # fresh state: the snapshot velocity is v
    set_particles(ctx, 0, cell, frac, v, w)
    E.efpi_deposit(ctx.ctx)
    c = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c)
    bits = E.efpi_sync(ctx.ctx, raise_on_error=False)
    assert bool(bits & E.DEV_WEIGHT) == flag


def test_restrict_state_matches_oracle():
    E = lib()
    spec = E.ReplicaSpec(512, 512.0, ppc=64, haar_levels=4)
    ctx = make_ctx([spec])
    parts = iaw_particles(spec, 13)
    set_particles(ctx, 0, *parts)
    c = ctx.new_coarse()
    E.efpi_restrict_state(ctx.ctx, c)
    got = c.view(2, -1).cpu().numpy()
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    x = x_of(parts[0], parts[1], g.h)
    ref = oefpi.restrict_state(x, parts[2].astype(np.float64), parts[3].astype(np.float64),
                               np.ones(x.size, bool), g, sch)
    assert metrics.rel_l2(got, ref) < 1e-7
    # after a plain PIC burst (half-step velocities re-centred with the current field)
    E.efpi_pic_burst(ctx.ctx, 7, False)
    E.efpi_restrict_state(ctx.ctx, c)
    got = c.view(2, -1).cpu().numpy()
    xp, vh, al, phi = opic.pic_run(x, parts[2].astype(np.float64), parts[3].astype(np.float64), g, 7)
    vi = vh + 0.5 * g.dt * opic.gather(opic.field(phi, g), xp, g)
    ref = oefpi.restrict_state(xp, vi, parts[3].astype(np.float64), al, g, sch)
    for m in range(2):
        assert metrics.rel_l2(got[m], ref[m]) < 1e-5


# ------------------------------------------------------------ absorbing walls --

def wall_particles(n_cells, seed, n_edge=4000, n_bulk=40000):
    """A bulk population in the middle (it makes the field) and ions in the two
    end cells moving out at 0.5 .. 3 cells per unit time, so that a step of
    dt = 0.1 takes a known part of them through x = 0 and x = L."""
    g = np.random.default_rng(seed)
    cb, fb, vb, wb = synth.random_particles(n_bulk, n_cells // 2, seed=seed, vth=0.2,
                                            w_mean=n_cells / (2.0 * n_bulk))
    cb = (cb + n_cells // 4).astype(np.int16)
    left = np.zeros(n_edge, np.int16)
    right = np.full(n_edge, n_cells - 1, np.int16)
    fe = g.random(2 * n_edge, dtype=np.float32) * np.float32(0.999)
    ve = g.uniform(0.5, 3.0, 2 * n_edge).astype(np.float32)
    ve[:n_edge] *= -1.0                                          # left end: towards x = 0
    we = (g.uniform(0.5, 1.5, 2 * n_edge) * 0.01).astype(np.float32)
    cell = np.concatenate([left, right, cb])
    order = np.argsort(cell, kind="stable")
    cat = lambda a, b: np.concatenate([a, b])[order]
    return (cell[order], cat(fe, fb), cat(ve, vb), cat(we, wb))


def test_one_step_through_both_walls():
    E = lib()
    n = 256
    spec = E.ReplicaSpec(n, float(n), bc=1, ppc=1, haar_levels=3, vth=0.1,
                         capacity=48000)
    ctx = make_ctx([spec])
    cell, frac, v, w = wall_particles(n, 41)
    set_particles(ctx, 0, cell, frac, v, w)
    E.efpi_deposit(ctx.ctx)
    E.efpi_solve_field(ctx.ctx, 80, cold=True)
    E.efpi_pic_burst(ctx.ctx, 1, False)
    gc, gf, gv, gw = particles_np(ctx)
    q, _, e = grid_np(ctx)
    g = oracle_grid(spec)
    x0 = x_of(cell, frac, g.h)
    alive0 = np.ones(x0.size, bool)
    _, phi0, e0 = opic.field_from_particles(x0, w.astype(np.float64), alive0, g)
    vh = v.astype(np.float64) + 0.5 * g.dt * opic.gather(e0, x0, g)
    x1, alive = opic.apply_bc(x0 + g.dt * vh, alive0, g)
    # both walls absorbed ions in this step, and exactly the oracle's ones
    assert np.sum(~alive & (x1 < 0)) > 100 and np.sum(~alive & (x1 >= g.length)) > 100
    assert np.array_equal(gc >= 0, alive)
    assert relmax(gv[alive], vh[alive]) < 1e-5
    assert np.max(np.abs(x_of(gc[alive], gf[alive], g.h) - x1[alive])) < 1e-5 * g.h
    # charge: survivors only, bit-exact, and the fused deposit equals the oracle's
    assert np.array_equal(q, opic.deposit_fx(gc, gf, gw, g))
    qsurv = int(np.sum(np.rint(w[alive].astype(np.float64) * 2.0 ** 40).astype(np.int64)))
    assert int(q.sum()) == qsurv


def test_burst_with_positions_moved_past_the_walls():
    # Plasma filling the box: over tau = Delta t - p dt of up to 20, the
    # co-evolving positions X + tau V of the outer ions leave [0, L) and are left
    # out of the snapshots (in flight to a wall), and ions reach the walls during
    # the burst itself.
    E = lib()
    n = 512
    spec = E.ReplicaSpec(n, float(n), bc=1, ppc=40, haar_levels=3, burst_steps=20,
                         macro_dt=20.0, vth=0.8)
    g, sch = oracle_grid(spec), oracle_scheme(spec)
    dens, u = synth.slab_profile(n, width=1.0)
    cell, frac, v, w = oefpi.load_particles(dens, u, g, sch, synth.lift_shift(43))
    parts = (cell.astype(np.int16), frac.astype(np.float32), v.astype(np.float32),
             w.astype(np.float32))
    gs, gn, os_, on = _burst_compare(spec, parts, "wide slab", newton_iters=3)
    # the exclusion acts: the first snapshot misses mass that left the box
    total = np.sum(w.astype(np.float64)) / g.h * 2.0 ** (-sch.levels / 2.0)
    assert np.sum(os_[0, 0]) < 0.98 * total
    assert abs(np.sum(gs[0, 0]) / np.sum(os_[0, 0]) - 1.0) < 2e-3
    # and ions were absorbed during the burst on both sides
    ctx = make_ctx([spec], newton_iters=3)
    set_particles(ctx, 0, *parts)
    E.efpi_pic_burst(ctx.ctx, spec.burst_steps, False)
    gc = particles_np(ctx)[0]
    assert np.sum(gc < 0) > 30
