"""Oracle fine solver with kinetic electrons, FP64.  TEST INFRASTRUCTURE ONLY
(see package header).

The paper's fine-scale model (Sec. 2, eq. 2.5; the two-species XES1 runs of
Sec. 4.1 and 4.2) moves electrons as particles too.  Units as oracle.pic
(length in Debye lengths, time in inverse ion plasma frequencies, potential in
T_e/e, density in n_0), so with mu = m_i / m_e the electrons have charge-to-mass
ratio -mu, plasma frequency sqrt(mu) and thermal speed sqrt(mu) at T_e.
Ions carry charge +w, electrons -w; the field solves the linear Poisson
equation -phi'' = n_i - n_e (eq. 2.2) on a periodic grid, with zero-mean phi.

At lifting (Sec. 3.3, the passive electron variables) the electrons are set to
the Boltzmann equilibrium of the lifted ions: phi solves the Poisson-Boltzmann
equation (eq. 3.15) for the ion density, n_e = exp(phi), V_e = V_i and
T_e = T_e0 (eq. 3.16), and they are loaded by the quiet start of App. C for
that shifted Maxwellian.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import efpi, pic
from .pic import Grid, PERIODIC

# The electron quiet start rotates its Hammersley points by the ion rotation of
# the same lift XOR this constant, so that the two species do not sample the
# same velocity quantiles in the same order.
ELECTRON_SHIFT_XOR = 0x9E3779B9


@dataclass
class Electrons:
    """Electron parameters of a kinetic replica."""

    mu: float = 1836.0        # m_i / m_e; charge-to-mass ratio -mu
    vth: float = 42.85        # thermal speed sqrt(T_e / m_e) in ion units (sqrt(mu) at T_e0)
    ppc: int = 100            # electrons per occupied cell at loading

    @property
    def qm(self) -> float:
        return -self.mu


def electron_shift(shift_i: int) -> int:
    return (int(shift_i) ^ ELECTRON_SHIFT_XOR) & 0xFFFFFFFF


# ----------------------------------------------------------------------------
# Field (eq. 2.2 with both species)
# ----------------------------------------------------------------------------

def net_charge_fx(ions, electrons, grid: Grid) -> np.ndarray:
    """Fixed-point node charge of both species: ion charge minus electron charge,
    each deposited by oracle.pic.deposit_fx (exact integer sums)."""
    return pic.deposit_fx(*ions, grid) - pic.deposit_fx(*electrons, grid)


def net_density(xi, wi, ai, xe, we, ae, grid: Grid) -> np.ndarray:
    """FP64 CIC node charge density n_i - n_e."""
    return (pic.deposit_density(xi[ai], wi[ai], grid)
            - pic.deposit_density(xe[ae], we[ae], grid))


def kinetic_field(xi, wi, ai, xe, we, ae, grid: Grid):
    """rho = n_i - n_e, phi from the linear Poisson equation, node field E."""
    assert grid.bc == PERIODIC
    rho = net_density(xi, wi, ai, xe, we, ae, grid)
    phi = pic.linear_poisson(rho, grid)
    return rho, phi, pic.field(phi, grid)


# ----------------------------------------------------------------------------
# Time stepping (eq. 2.5 for both species, leapfrog)
# ----------------------------------------------------------------------------

def species_step(x, v_half, alive, qm: float, e_nodes, grid: Grid):
    """v^{n+1/2} = v^{n-1/2} + (q/m) dt E(x^n);  x^{n+1} = x^n + dt v^{n+1/2}; periodic wrap."""
    v_new = v_half.copy()
    x_new = x.copy()
    v_new[alive] = v_half[alive] + qm * grid.dt * pic.gather(e_nodes, x[alive], grid)
    x_new[alive] = x[alive] + grid.dt * v_new[alive]
    x_new, alive = pic.apply_bc(x_new, alive, grid)
    return x_new, v_new, alive


def kinetic_run(ions, electrons, grid: Grid, el: Electrons, steps: int):
    """Plain two-species PIC from integer-time velocities.

    ions, electrons: (x, v, w) FP64 arrays.  The leapfrog starts with the half
    step back v^{-1/2} = v^0 - (q/m) dt/2 E^0 of each species.  Returns
    ((x_i, vh_i), (x_e, vh_e), phi) after `steps` steps, velocities at the last
    half step.
    """
    xi, vi, wi = (np.array(a, dtype=np.float64) for a in ions)
    xe, ve, we = (np.array(a, dtype=np.float64) for a in electrons)
    ai = np.ones(xi.size, bool)
    ae = np.ones(xe.size, bool)
    _, phi, e = kinetic_field(xi, wi, ai, xe, we, ae, grid)
    vi = vi - 0.5 * grid.dt * pic.gather(e, xi, grid)
    ve = ve - el.qm * 0.5 * grid.dt * pic.gather(e, xe, grid)
    for _ in range(steps):
        xi, vi, ai = species_step(xi, vi, ai, 1.0, e, grid)
        xe, ve, ae = species_step(xe, ve, ae, el.qm, e, grid)
        _, phi, e = kinetic_field(xi, wi, ai, xe, we, ae, grid)
    return (xi, vi), (xe, ve), phi


def momentum(vi, wi, ve, we, el: Electrons) -> float:
    """Total momentum: ion mass w per ion, electron mass w / mu per electron."""
    return float(np.sum(wi * vi) + np.sum(we * ve) / el.mu)


# ----------------------------------------------------------------------------
# Electron loading (Sec. 3.3 passive variables; App. C quiet start)
# ----------------------------------------------------------------------------

def load_electrons(n_nodes, u_nodes, grid: Grid, el: Electrons, shift: int, n_floor=1e-6):
    """Quiet-start electrons for node profiles n_e, u_e: the ion loader of
    oracle.efpi (App. C) with the electron count and thermal speed."""
    sch = efpi.Scheme(ppc=el.ppc, vth=el.vth, n_floor=n_floor)
    return efpi.load_particles(n_nodes, u_nodes, grid, sch, shift)


def boltzmann_electrons(x_i, w_i, u_nodes, grid: Grid, el: Electrons, shift: int, n_floor=1e-6):
    """Electrons in Boltzmann equilibrium with the given ions: phi from eq. 3.15
    (Newton to 1e-12) for the ion density, then n_e = exp(phi) and u_e = u_nodes
    (eq. 3.16).  Returns (cell, frac, v, w, phi)."""
    rho_i = pic.deposit_density(x_i, w_i, grid)
    phi, _, ok = pic.newton_poisson(rho_i, grid, max_iter=200)
    if not ok:
        raise RuntimeError("oracle Newton did not converge")
    c, f, v, w = load_electrons(np.exp(phi), u_nodes, grid, el, shift, n_floor)
    return c, f, v, w, phi


def reset_electrons(x_i, vc_i, w_i, grid: Grid, el: Electrons, shift: int, n_floor=1e-6):
    """Electrons reset to the Boltzmann equilibrium of the current ions (the
    control run of Sec. 4.1): ion node density and momentum by CIC, mean velocity
    u = j / n where n > n_floor (else 0), then boltzmann_electrons with that u.
    vc_i are the ions' time-centred velocities.  Returns (cell, frac, v, w, phi)."""
    n = pic.deposit_density(x_i, w_i, grid)
    j = pic.deposit_mass(x_i, w_i * vc_i, grid) / grid.node_volume()
    u = np.zeros_like(n)
    ok = n > n_floor
    u[ok] = j[ok] / n[ok]
    return boltzmann_electrons(x_i, w_i, u, grid, el, shift, n_floor)


# ----------------------------------------------------------------------------
# The projective cycle with kinetic electrons (Sec. 3.1, App. B)
# ----------------------------------------------------------------------------

def kinetic_burst(ions, electrons, grid: Grid, sch: efpi.Scheme, el: Electrons, steps=None):
    """Two-species burst with restriction of the ions after every step.

    As oracle.efpi.pic_burst: E_n is the field at the burst start, snapshot p
    restricts the ions' time-centred velocities with tau = Delta t - p dt along
    the co-evolving frame, then both species take a leapfrog step.  Returns the
    snapshots (N_e + 1, 2, N_c)."""
    ne = sch.burst_steps if steps is None else steps
    xi, vi, wi = (np.array(a, dtype=np.float64) for a in ions)
    xe, ve, we = (np.array(a, dtype=np.float64) for a in electrons)
    ai = np.ones(xi.size, bool)
    ae = np.ones(xe.size, bool)
    _, phi, e = kinetic_field(xi, wi, ai, xe, we, ae, grid)
    e_n = e.copy()
    vi = vi - 0.5 * grid.dt * pic.gather(e, xi, grid)
    ve = ve - el.qm * 0.5 * grid.dt * pic.gather(e, xe, grid)
    snaps = []
    for p in range(ne + 1):
        vp = vi[ai] + 0.5 * grid.dt * pic.gather(e, xi[ai], grid)
        tau = sch.macro_dt - p * grid.dt
        snaps.append(efpi.restrict_snapshot(xi[ai], vp, pic.gather(e_n, xi[ai], grid), wi[ai],
                                            tau, grid, sch.levels, sch.coevolving))
        if p < ne:
            xi, vi, ai = species_step(xi, vi, ai, 1.0, e, grid)
            xe, ve, ae = species_step(xe, ve, ae, el.qm, e, grid)
            _, phi, e = kinetic_field(xi, wi, ai, xe, we, ae, grid)
    return np.array(snaps)


def kinetic_lift(coarse, grid: Grid, sch: efpi.Scheme, el: Electrons, shift: int):
    """Ions by the lift of oracle.efpi (profile, quiet start, block correction),
    then Boltzmann electrons for them with the ions' fine velocity profile.
    Returns (ions (x, v, w), electrons (x, v, w))."""
    ci, fi, vi, wi = efpi.lift(coarse, grid, sch, shift)
    xi = efpi.particles_to_x(ci, fi, grid)
    n_f, j_f = efpi.lift_profile(coarse, grid, sch)
    u_f = efpi.velocity_profile(n_f, j_f, sch)
    ce, fe, ve, we, _ = boltzmann_electrons(xi, wi, u_f, grid, el, electron_shift(shift),
                                            sch.n_floor)
    xe = efpi.particles_to_x(ce, fe, grid)
    return (xi, vi, wi), (xe, ve, we)


def kinetic_macro_step(coarse, grid: Grid, sch: efpi.Scheme, el: Electrons, shift: int):
    """One EFPI macro step with kinetic electrons: lift both species, burst with
    ion restriction, least squares and projection (eqs. 3.17-3.18)."""
    ions, electrons = kinetic_lift(coarse, grid, sch, el, shift)
    snaps = kinetic_burst(ions, electrons, grid, sch, el)
    return efpi.project(snaps, grid.dt, sch.macro_dt), snaps
