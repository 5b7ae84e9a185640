"""Pins of the kinetic-electron oracle against invariants and dispersion relations.

Each check uses a result fixed by the mathematics: exact momentum conservation
of the centred-field CIC scheme with both species, the cold two-species plasma
frequency through the leapfrog dispersion relation, global neutrality of the
Boltzmann equilibrium on a periodic grid, and the exact weight sums of the
quiet start.
"""
import numpy as np
import pytest

import synth
from oracle import efpi, kinetic, pic
from oracle.kinetic import Electrons
from oracle.pic import Grid


def _species(n_cells, ppc, seed, vth, shift_u=0.0):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, n_cells, n_cells * ppc)
    v = shift_u + vth * rng.standard_normal(x.size)
    w = (1.0 + 0.2 * rng.uniform(-1, 1, x.size)) / ppc
    return x, v, w


def test_kinetic_momentum_conserved_exactly():
    # P = sum w v_i + sum w v_e / mu changes per step by dt sum_k rho_k E_k h, which is
    # zero for the centred field of the discrete Poisson solution (the sum telescopes).
    g = Grid(64, 64.0, dt=0.02)
    el = Electrons(mu=50.0, vth=7.0, ppc=20)
    ions = _species(64, 20, 1, 0.3, 0.1)
    electrons = _species(64, 20, 2, el.vth)
    (xi, vi), (xe, ve), _ = kinetic.kinetic_run(ions, electrons, g, el, 1)
    p0 = kinetic.momentum(vi, ions[2], ve, electrons[2], el)
    scale = np.sum(np.abs(ions[2] * vi)) + np.sum(np.abs(electrons[2] * ve)) / el.mu
    (xi, vi), (xe, ve), _ = kinetic.kinetic_run(ions, electrons, g, el, 40)
    p1 = kinetic.momentum(vi, ions[2], ve, electrons[2], el)
    assert abs(p1 - p0) < 1e-12 * scale


def test_kinetic_momentum_detects_a_wrong_sign():
    # the same run with the electron force sign flipped must not conserve momentum
    g = Grid(64, 64.0, dt=0.02)
    el = Electrons(mu=50.0, vth=7.0, ppc=20)
    bad = Electrons(mu=-50.0, vth=7.0, ppc=20)
    ions = _species(64, 20, 1, 0.3, 0.1)
    electrons = _species(64, 20, 2, el.vth)
    (_, vi0), (_, ve0), _ = kinetic.kinetic_run(ions, electrons, g, bad, 1)
    (_, vi1), (_, ve1), _ = kinetic.kinetic_run(ions, electrons, g, bad, 40)
    m = lambda vi, ve: np.sum(ions[2] * vi) + np.sum(electrons[2] * ve) / el.mu
    scale = np.sum(np.abs(ions[2] * vi0)) + np.sum(np.abs(electrons[2] * ve0)) / el.mu
    assert abs(m(vi1, ve1) - m(vi0, ve0)) > 1e-6 * scale


def test_cold_two_species_plasma_frequency():
    # Cold ions and electrons, electrons displaced by a small mode: the charge
    # oscillates at omega^2 = omega_pe^2 + omega_pi^2 = mu + 1 (cold two-fluid
    # theory), seen through the leapfrog relation sin(omega dt / 2) = (dt / 2) omega_p.
    n, ppc, mode, amp = 64, 16, 1, 0.01
    mu = 24.0
    g = Grid(n, float(n), dt=0.02)
    el = Electrons(mu=mu, vth=0.0, ppc=ppc)
    x0 = (np.arange(n * ppc) + 0.5) / ppc
    k = 2 * np.pi * mode / n
    xi = x0.copy()
    xe = np.mod(x0 - (amp / k) * np.sin(k * x0), n)
    w = np.full(x0.size, 1.0 / ppc)
    zeros = np.zeros_like(x0)
    ai = np.ones(x0.size, bool)
    _, phi, e = kinetic.kinetic_field(xi, w, ai, xe, w, ai, g)
    vi = zeros - 0.5 * g.dt * pic.gather(e, xi, g)
    ve = zeros - el.qm * 0.5 * g.dt * pic.gather(e, xe, g)
    xk = np.arange(n)
    amps = []
    steps = 160
    for _ in range(steps):
        rho = kinetic.net_density(xi, w, ai, xe, w, ai, g)
        amps.append(np.sum(rho * np.cos(k * xk)) * 2 / n)
        xi, vi, ai = kinetic.species_step(xi, vi, ai, 1.0, e, g)
        xe, ve, ai2 = kinetic.species_step(xe, ve, ai, el.qm, e, g)
        _, phi, e = kinetic.kinetic_field(xi, w, ai, xe, w, ai2, g)
    a = np.array(amps)
    t = np.arange(steps) * g.dt
    zc = [i for i in range(1, steps) if np.sign(a[i]) != np.sign(a[i - 1])]
    cross = [t[i - 1] + (t[i] - t[i - 1]) * a[i - 1] / (a[i - 1] - a[i]) for i in zc]
    w_num = np.pi / np.mean(np.diff(cross))
    w_leap = 2.0 / g.dt * np.arcsin(0.5 * g.dt * np.sqrt(mu + 1.0))
    assert len(cross) >= 4
    assert abs(w_num / w_leap - 1.0) < 0.01


def test_boltzmann_electrons_neutral_and_in_equilibrium():
    # Summing -phi'' + exp(phi) = n_i over a periodic grid removes the Laplacian, so
    # the electron node charge sum equals the ion one; the quiet start's weights sum
    # per cell to h (n_l + n_r) / 2, so the electron weights total the ion charge.
    n = 128
    g = Grid(n, float(n))
    sch = efpi.Scheme(ppc=32, vth=0.3)
    dens, u = synth.iaw_profile(n, float(n))
    ci, fi, vi, wi = efpi.load_particles(dens, u, g, sch, synth.lift_shift(4))
    xi = efpi.particles_to_x(ci, fi, g)
    el = Electrons(mu=100.0, vth=10.0, ppc=24)
    ce, fe, ve, we, phi = kinetic.boltzmann_electrons(xi, wi, u, g, el, 77)
    rho_i = pic.deposit_density(xi, wi, g)
    assert np.max(np.abs(pic.neg_laplacian(g) @ phi + np.exp(phi) - rho_i)) < 1e-10
    assert np.sum(we) == pytest.approx(np.sum(wi), rel=1e-7)
    # weights are exp(phi) interpolated at the electron, times h / ppc
    right = (ce + 1) % n
    want = ((1 - fe) * np.exp(phi[ce]) + fe * np.exp(phi[right])) * g.h / el.ppc
    assert np.max(np.abs(we - want)) < 1e-14
    # velocities: the ion mean-velocity profile plus the electron thermal spread
    ux = (1 - fe) * u[ce] + fe * u[right]
    z = (ve - ux) / el.vth
    assert abs(np.mean(z)) < 0.02 and abs(np.std(z) - 1.0) < 0.02


def test_electron_shift_differs_from_ion_shift():
    for s in (0, 1, 0xFFFFFFFF, synth.lift_shift(9)):
        e = kinetic.electron_shift(s)
        assert 0 <= e < 2 ** 32 and e != s and kinetic.electron_shift(e) == s


def test_kinetic_burst_snapshots_are_restrictions_of_the_plain_run():
    # Without the co-evolving frame, snapshot p is the plain restriction of the
    # ions after p two-species steps with time-centred velocities.
    n = 64
    g = Grid(n, float(n), dt=0.02)
    sch = efpi.Scheme(levels=2, burst_steps=6, macro_dt=1.0, coevolving=False, ppc=16)
    el = Electrons(mu=30.0, vth=5.5, ppc=16)
    ions = _species(n, 16, 5, 0.3)
    electrons = _species(n, 16, 6, el.vth)
    snaps = kinetic.kinetic_burst(ions, electrons, g, sch, el)
    for p in (0, 3, 6):
        (xi, vh), (xe, _), phi = kinetic.kinetic_run(ions, electrons, g, el, p)
        vc = vh + 0.5 * g.dt * pic.gather(pic.field(phi, g), xi, g)
        ref = efpi.restrict_state(xi, vc, ions[2], np.ones(xi.size, bool), g, sch)
        assert np.max(np.abs(snaps[p] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_reset_velocity_profile_is_the_ion_mean_velocity():
    # Ions drifting as a block at velocity U: the node momentum over the node
    # density is U exactly wherever there are ions, so the reset electrons carry
    # mean velocity U (their quiet-start deviates have zero mean per cell pair).
    n, ppc = 64, 40
    g = Grid(n, float(n))
    rng = np.random.default_rng(3)
    xi = rng.uniform(0, n, n * ppc)
    wi = rng.uniform(0.5, 1.5, xi.size) / ppc
    U = 0.37
    el = Electrons(mu=100.0, vth=10.0, ppc=32)
    c, f, v, w, phi = kinetic.reset_electrons(xi, np.full(xi.size, U), wi, g, el, 5)
    right = (c + 1) % n
    rho = pic.deposit_density(xi, wi, g)
    j = pic.deposit_mass(xi, wi * U, g) / g.node_volume()
    assert np.max(np.abs(j / rho - U)) < 1e-14
    z = (v - U) / el.vth
    assert abs(np.mean(z)) < 0.01 and abs(np.std(z) - 1.0) < 0.02
    # electron weights are exp(phi) at the electron, phi solving eq. 3.15 for the ions
    assert np.max(np.abs(pic.neg_laplacian(g) @ phi + np.exp(phi) - rho)) < 1e-10
    want = ((1 - f) * np.exp(phi[c]) + f * np.exp(phi[right])) * g.h / el.ppc
    assert np.max(np.abs(w - want)) < 1e-14
