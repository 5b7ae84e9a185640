"""Oracle fine-scale solver: electrostatic 1D1V PIC for kinetic ions with
Boltzmann electrons, in FP64.  TEST INFRASTRUCTURE ONLY (see package header).

Units (Sec. 2.1, eq. 2.3 and the rescaled eq. 3.15): length in Debye lengths,
time in inverse ion plasma frequencies, potential in T_e/e, density in n_0.
The ion charge-to-mass ratio is 1, the equations of motion are dX/dt = V,
dV/dt = E = -dphi/dx (eq. 2.5), and the field equation with Boltzmann
electrons (eqs. 3.2, 3.14-3.16) is  -phi'' + exp(phi) = n_i.

Grid: nodes x_k = k h.  Periodic domains have N nodes (node N is node 0);
absorbing-wall domains have N + 1 nodes and the two wall nodes own half a cell.
A particle in cell c = floor(x / h) with offset theta = x / h - c shares its
weight (1 - theta) w to node c and theta w to node c + 1 (the CIC weighting of
Sec. 2.2 with the hat function of Sec. 3.3; the update rule of App. B).

Closures: 0 = Boltzmann electrons solved by Newton's method (eq. 3.15, Sec. 3.3),
1 = fixed neutralising background (linear Poisson eq. 2.2, periodic only; test
closure), 2 = no field (E = 0; test closure for free streaming).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

PERIODIC = 0
WALLS = 1

BOLTZMANN = 0
LINEAR = 1
NOFIELD = 2

FX_SCALE = 2.0 ** 40  # fixed-point unit of charge: 2^-40


@dataclass
class Grid:
    """One replica's grid and time-step parameters."""

    n_cells: int
    length: float
    bc: int = PERIODIC
    closure: int = BOLTZMANN
    dt: float = 0.1

    @property
    def h(self) -> float:
        return self.length / self.n_cells

    @property
    def n_nodes(self) -> int:
        return self.n_cells if self.bc == PERIODIC else self.n_cells + 1

    def node_volume(self) -> np.ndarray:
        vol = np.full(self.n_nodes, self.h)
        if self.bc == WALLS:
            vol[0] = vol[-1] = 0.5 * self.h
        return vol


# ----------------------------------------------------------------------------
# Charge deposition (Sec. 2.2; weights of App. B)
# ----------------------------------------------------------------------------

def deposit_fx(cell, frac, w, grid: Grid) -> np.ndarray:
    """Fixed-point CIC charge of FP32 particles: int64 node charges in 2^-40 units.

    The particle weight is quantised as q = rint(w * 2^40); the right-node share
    is q_R = rint(theta * q) with theta the FP32 in-cell offset, and the left
    share is q - q_R, so every particle deposits exactly q (charge conservation
    holds exactly, whatever the summation order).  Products are IEEE binary64
    with round-to-nearest-even.  Dead particles (cell < 0) deposit nothing.
    """
    cell = np.asarray(cell).astype(np.int64)
    frac = np.asarray(frac, dtype=np.float32).astype(np.float64)
    w = np.asarray(w, dtype=np.float32).astype(np.float64)
    alive = cell >= 0
    cell, frac, w = cell[alive], frac[alive], w[alive]
    q = np.rint(w * FX_SCALE).astype(np.int64)
    q_right = np.rint(frac * q.astype(np.float64)).astype(np.int64)
    q_left = q - q_right
    right = cell + 1
    if grid.bc == PERIODIC:
        right = right % grid.n_cells
    out = np.zeros(grid.n_nodes, dtype=np.int64)
    np.add.at(out, cell, q_left)
    np.add.at(out, right, q_right)
    return out


def fx_to_density(q_fx, grid: Grid) -> np.ndarray:
    """Node density rho_k = Q_k 2^-40 / V_k from fixed-point node charges."""
    return np.asarray(q_fx, dtype=np.float64) / FX_SCALE / grid.node_volume()


def cic_nodes(x, grid: Grid):
    """Cell index and in-cell offset of absolute positions x (FP64)."""
    s = np.asarray(x, dtype=np.float64) / grid.h
    c = np.floor(s)
    theta = s - c
    c = c.astype(np.int64)
    return c, theta


def deposit_mass(x, weight, grid: Grid) -> np.ndarray:
    """FP64 CIC deposit of arbitrary per-particle weights: node masses (not densities)."""
    c, theta = cic_nodes(x, grid)
    right = c + 1
    if grid.bc == PERIODIC:
        c = c % grid.n_cells
        right = right % grid.n_cells
    out = np.zeros(grid.n_nodes)
    out += np.bincount(c, weights=(1.0 - theta) * weight, minlength=grid.n_nodes)[: grid.n_nodes]
    out += np.bincount(right, weights=theta * weight, minlength=grid.n_nodes)[: grid.n_nodes]
    return out


def deposit_density(x, w, grid: Grid) -> np.ndarray:
    """FP64 CIC ion density rho_k = (sum of shares) / V_k."""
    return deposit_mass(x, w, grid) / grid.node_volume()


# ----------------------------------------------------------------------------
# Field solve (eq. 3.15 by Newton's method; eq. 2.2 for the linear closure)
# ----------------------------------------------------------------------------

def neg_laplacian(grid: Grid) -> sp.csr_matrix:
    """Matrix of -phi'' by second differences.

    Periodic: cyclic.  Walls: the Neumann condition phi' = 0 through a mirrored
    ghost node, i.e. row 0 reads -2 (phi_1 - phi_0) / h^2 and row N likewise.
    """
    n = grid.n_nodes
    h2 = grid.h * grid.h
    main = np.full(n, 2.0 / h2)
    off = np.full(n - 1, -1.0 / h2)
    a = sp.diags([off, main, off], [-1, 0, 1], shape=(n, n), format="lil")
    if grid.bc == PERIODIC:
        a[0, n - 1] = -1.0 / h2
        a[n - 1, 0] = -1.0 / h2
    else:
        a[0, 1] = -2.0 / h2
        a[n - 1, n - 2] = -2.0 / h2
    return a.tocsr()


def newton_poisson(rho, grid: Grid, phi0=None, tol=1e-12, max_iter=60):
    """Solve -phi'' + exp(phi) = rho (eq. 3.15) by damped Newton iteration.

    Returns (phi, iterations, converged).  Start: phi0 if given, else
    ln(max(rho, 1e-8)) (the quasineutral potential of eq. 3.4 as first guess).
    Each step solves J delta = -F with J = A + diag(exp(phi)) by a sparse direct
    solve, caps |delta| at 2 per component and halves the step while the
    residual norm grows.  Converged when max|delta| <= tol.
    """
    rho = np.asarray(rho, dtype=np.float64)
    a = neg_laplacian(grid)
    phi = np.log(np.maximum(rho, 1e-8)) if phi0 is None else np.array(phi0, dtype=np.float64)

    def resid(p):
        return a @ p + np.exp(p) - rho

    f = resid(phi)
    for it in range(1, max_iter + 1):
        jac = (a + sp.diags(np.exp(phi))).tocsc()
        delta = spla.spsolve(jac, -f)
        delta = np.clip(delta, -2.0, 2.0)
        step = 1.0
        fn = np.linalg.norm(f)
        while True:
            trial = phi + step * delta
            ft = resid(trial)
            if np.linalg.norm(ft) <= fn or step < 1e-4:
                break
            step *= 0.5
        phi, f = trial, ft
        if np.max(np.abs(step * delta)) <= tol:
            return phi, it, True
    return phi, max_iter, False


def linear_poisson(rho, grid: Grid):
    """Solve -phi'' = rho - mean(rho) with mean(phi) = 0 (eq. 2.2, periodic).

    The cyclic matrix is singular (constants); pin phi_0 = 0, solve the
    remaining nonsingular system directly, then remove the mean.
    """
    assert grid.bc == PERIODIC
    rho = np.asarray(rho, dtype=np.float64)
    a = neg_laplacian(grid).tocsc()
    rhs = rho - rho.mean()
    sub = a[1:, 1:]
    phi = np.zeros_like(rhs)
    phi[1:] = spla.spsolve(sub, rhs[1:])
    return phi - phi.mean()


def solve_field(rho, grid: Grid, phi0=None):
    """Potential for the grid's closure."""
    if grid.closure == BOLTZMANN:
        phi, _, ok = newton_poisson(rho, grid, phi0, max_iter=200)
        if not ok:
            raise RuntimeError("oracle Newton did not converge")
        return phi
    if grid.closure == LINEAR:
        return linear_poisson(rho, grid)
    return np.zeros(grid.n_nodes)


def field(phi, grid: Grid) -> np.ndarray:
    """Node field E_k = -(phi_{k+1} - phi_{k-1}) / (2h); E = 0 on walls."""
    phi = np.asarray(phi, dtype=np.float64)
    if grid.bc == PERIODIC:
        return -(np.roll(phi, -1) - np.roll(phi, 1)) / (2.0 * grid.h)
    e = np.zeros_like(phi)
    e[1:-1] = -(phi[2:] - phi[:-2]) / (2.0 * grid.h)
    return e


def gather(e_nodes, x, grid: Grid) -> np.ndarray:
    """Field at particle positions with the deposit's CIC weights."""
    c, theta = cic_nodes(x, grid)
    right = c + 1
    if grid.bc == PERIODIC:
        c = c % grid.n_cells
        right = right % grid.n_cells
    return (1.0 - theta) * e_nodes[c] + theta * e_nodes[right]


# ----------------------------------------------------------------------------
# Time stepping (eq. 2.5, leapfrog)
# ----------------------------------------------------------------------------

def apply_bc(x, alive, grid: Grid):
    """Periodic wrap, or absorption of particles that left [0, L)."""
    if grid.bc == PERIODIC:
        return np.mod(x, grid.length), alive
    out = (x < 0.0) | (x >= grid.length)
    return x, alive & ~out


def leapfrog_step(x, v_half, w, alive, e_nodes, grid: Grid):
    """One leapfrog step: v^{n+1/2} = v^{n-1/2} + dt E(x^n); x^{n+1} = x^n + dt v^{n+1/2}."""
    v_new = v_half.copy()
    x_new = x.copy()
    ep = gather(e_nodes, x[alive], grid)
    v_new[alive] = v_half[alive] + grid.dt * ep
    x_new[alive] = x[alive] + grid.dt * v_new[alive]
    x_new, alive = apply_bc(x_new, alive, grid)
    return x_new, v_new, alive


def field_from_particles(x, w, alive, grid: Grid, phi0=None):
    rho = deposit_density(x[alive], w[alive], grid)
    phi = solve_field(rho, grid, phi0)
    return rho, phi, field(phi, grid)


def pic_run(x, v, w, grid: Grid, steps: int, alive=None, phi0=None):
    """Plain PIC: `steps` leapfrog steps from integer-time velocities v.

    The first half step back v^{-1/2} = v^0 - dt/2 E^0 starts the leapfrog.
    Returns positions, half-step velocities, alive mask and the last potential.
    """
    x = np.array(x, dtype=np.float64)
    w = np.array(w, dtype=np.float64)
    alive = np.ones(x.shape, bool) if alive is None else np.array(alive)
    _, phi, e = field_from_particles(x, w, alive, grid, phi0)
    vh = np.array(v, dtype=np.float64)
    vh[alive] -= 0.5 * grid.dt * gather(e, x[alive], grid)
    for _ in range(steps):
        x, vh, alive = leapfrog_step(x, vh, w, alive, e, grid)
        _, phi, e = field_from_particles(x, w, alive, grid, phi)
    return x, vh, alive, phi


# ----------------------------------------------------------------------------
# Diagnostics
# ----------------------------------------------------------------------------

def energy(x, v, w, alive, phi, grid: Grid) -> float:
    """Total energy of ions plus Boltzmann electrons and field.

    W = sum_j w_j v_j^2 / 2 + sum_edges h (dphi/h)^2 / 2 + sum_k V_k (phi_k - 1) e^{phi_k}.
    For -phi'' + e^phi = n the field part changes at the rate int phi dn/dt, which
    is minus the work on the ions, so W is the conserved energy of the
    Boltzmann-electron model (the paper does not state it).
    """
    kin = 0.5 * np.sum(w[alive] * v[alive] ** 2)
    if grid.bc == PERIODIC:
        dphi = np.roll(phi, -1) - phi
    else:
        dphi = phi[1:] - phi[:-1]
    fld = 0.5 * np.sum(dphi ** 2) / grid.h
    pot = np.sum(grid.node_volume() * (phi - 1.0) * np.exp(phi))
    return kin + fld + pot


def momentum(v, w, alive) -> float:
    """Total ion momentum sum w v (its relative change is what Sec. 4.1 plots)."""
    return float(np.sum(w[alive] * v[alive]))
