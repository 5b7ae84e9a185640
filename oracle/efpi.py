"""Oracle coarse representation and projective cycle, FP64.
TEST INFRASTRUCTURE ONLY (see package header).

Coarse variables: the Haar scaling coefficients, `levels` levels below the
fine grid, of the ion density and of the ion momentum density (the spatial
analogue of the wavelet coarsening of Sec. 3.3 and App. A, applied to the
density and momentum moments).  Each coefficient is
c_B = 2^{-l/2} sum_{k in B} M_k / h, with M_k the CIC node mass of block B's
nodes, which is what l levels of the orthonormal fast Haar transform give.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.special import ndtri

from . import pic
from .pic import Grid, PERIODIC, WALLS


@dataclass
class Scheme:
    """Projective-integration parameters of one replica."""

    levels: int = 4          # l: Haar levels between fine nodes and coarse blocks
    burst_steps: int = 20    # N_e fine steps per macro step (Sec. 3.1)
    macro_dt: float = 20.0   # Delta t (Sec. 3.1, eq. 3.17)
    coevolving: bool = True  # restriction along approximate characteristics (App. B)
    ppc: int = 100           # ions per occupied cell at lifting
    vth: float = 0.316227766016838  # sqrt(T_i / T_e) of the lifted Maxwellian
    lift_linear: bool = True  # linear interpolation of block means (else piecewise constant)
    n_floor: float = 1e-6    # density below which a cell is empty
    moments: int = 2         # 2: density and momentum; 3: and the second velocity
                             # moment (the EFREE variables n, V, P of Sec. 3.2)


# ----------------------------------------------------------------------------
# Haar transform (App. A: fast DWT with the Haar filters)
# ----------------------------------------------------------------------------

def haar_analysis(f, levels: int):
    """l levels of the orthonormal fast Haar transform of f (length divisible by 2^l).

    Returns (scaling coefficients at the coarse level, list of detail arrays
    from fine to coarse).
    """
    s = np.asarray(f, dtype=np.float64)
    details = []
    for _ in range(levels):
        even, odd = s[0::2], s[1::2]
        details.append((even - odd) / np.sqrt(2.0))
        s = (even + odd) / np.sqrt(2.0)
    return s, details


def haar_synthesis(s, details):
    """Inverse of haar_analysis."""
    s = np.asarray(s, dtype=np.float64)
    for d in reversed(details):
        out = np.empty(2 * s.size)
        out[0::2] = (s + d) / np.sqrt(2.0)
        out[1::2] = (s - d) / np.sqrt(2.0)
        s = out
    return s


def fold_nodes(node_values, grid: Grid):
    """Node array of length N: on walls the last node N joins the last block."""
    v = np.asarray(node_values, dtype=np.float64)
    if grid.bc == WALLS:
        v = v[:-1].copy()
        v[-1] += node_values[-1]
    return v


# ----------------------------------------------------------------------------
# Restriction with the co-evolving frame (Sec. 3.3, App. B eqs. B.4-B.5)
# ----------------------------------------------------------------------------

def restrict_snapshot(x, v_p, e_n_at_x, w, tau, grid: Grid, levels: int, coevolving=True,
                      moments: int = 2):
    """Coarse (density, momentum[, second moment]) coefficients of one snapshot,
    shape (moments, N_c).

    Each particle is moved along the approximate characteristic of eq. B.4 over
    the remaining time tau = Delta t - p dt: X~ = X + tau V, V~ = V + tau E_n(X),
    with E_n the field stored when the burst started.  Its weight w and its
    momentum w V~ are deposited with CIC weights at X~ (eq. B.5; the velocity
    histogram of the paper is replaced by its first velocity moments), and the
    node masses are coarsened by the fast Haar transform.  With moments = 3 the
    second moment w V~^2 is deposited the same way: n, nV and nV^2 + P carry the
    EFREE variables n, V and P (Sec. 3.2) in a form linear in the particles.  On
    walls, a particle whose X~ lies outside [0, L) is left out of the snapshot.
    With coevolving=False, tau = 0 (the plain deposition of Table 2).
    """
    x = np.asarray(x, dtype=np.float64)
    if coevolving:
        xt = x + tau * v_p
        vt = v_p + tau * e_n_at_x
    else:
        xt, vt = x.copy(), np.asarray(v_p, dtype=np.float64)
    if grid.bc == PERIODIC:
        xt = np.mod(xt, grid.length)
        keep = np.ones(xt.shape, bool)
    else:
        keep = (xt >= 0.0) & (xt < grid.length)
    out = np.empty((moments, grid.n_cells >> levels))
    for m, weight in enumerate((w, w * vt, w * vt * vt)[:moments]):
        mass = pic.deposit_mass(xt[keep], np.asarray(weight)[keep], grid)
        out[m], _ = haar_analysis(fold_nodes(mass, grid) / grid.h, levels)
    return out


# ----------------------------------------------------------------------------
# Least-squares slope and projection (eqs. 3.17-3.18)
# ----------------------------------------------------------------------------

def ls_slope(snaps, dt: float):
    """Time derivative of the coarse variables by the estimator of eq. 3.18.

    snaps[p] holds the snapshot after p fine steps, p = 0..N_e.  The index of
    the weight (printed as i) is read as the summation index p; with that
    reading the formula is the ordinary least-squares slope.
    """
    snaps = np.asarray(snaps, dtype=np.float64)
    ne = snaps.shape[0] - 1
    acc = np.zeros(snaps.shape[1:])
    for p in range(ne // 2 + 1):
        coef = 6.0 * (ne - 2 * p) / (ne * (ne + 1) * (ne + 2) * dt)
        acc += coef * (snaps[ne - p] - snaps[p])
    return acc


def project(snaps, dt: float, macro_dt: float):
    """Forward-Euler projective step from the last snapshot (eq. 3.17)."""
    snaps = np.asarray(snaps, dtype=np.float64)
    ne = snaps.shape[0] - 1
    return snaps[ne] + (macro_dt - ne * dt) * ls_slope(snaps, dt)


def project2(snaps, dt: float, macro_dt: float, slope_prev=None, gap=None):
    """Second-order projective step (the higher-order projection mentioned after
    eq. 3.17), read as Adams-Bashforth 2 on the burst slopes.

    The LS slope f of this burst (eq. 3.18) estimates the derivative at the
    burst's centre; slope_prev estimates it at the previous burst's centre, gap
    (the previous Delta t) earlier.  Their linear extrapolation to the middle of
    the leap [N_e dt, Delta t] is f* = f + (f - f_prev) Delta t / (2 gap), and the
    state advances from the last snapshot by (Delta t - N_e dt) f*.  Returns
    (f, forward-Euler projection of eq. 3.17, second-order projection); without
    slope_prev the second-order step is the Euler step.
    """
    snaps = np.asarray(snaps, dtype=np.float64)
    ne = snaps.shape[0] - 1
    f = ls_slope(snaps, dt)
    leap = macro_dt - ne * dt
    euler = snaps[ne] + leap * f
    if slope_prev is None:
        return f, euler, euler.copy()
    fstar = f + (f - np.asarray(slope_prev, dtype=np.float64)) * (macro_dt / (2.0 * gap))
    return f, euler, snaps[ne] + leap * fstar


def next_macro_dt(macro_dt: float, err: float, tol: float, dt_min: float, dt_max: float,
                  safety: float = 0.9) -> float:
    """Step-size rule of the adaptive projective integrator.

    err (eq. 4.2 between the second-order and the Euler projections of the
    coarse density) estimates the local error of a first-order step, which grows
    as Delta t^2, so the next step is Delta t (tol / err)^{1/2} times a safety
    factor, changed by at most a factor 2 either way and kept in [dt_min, dt_max].
    """
    factor = 2.0 if err <= 0.0 else min(2.0, max(0.5, safety * np.sqrt(tol / err)))
    return float(min(dt_max, max(dt_min, macro_dt * factor)))


# ----------------------------------------------------------------------------
# Lifting: coarse coefficients -> fine profile -> quiet-start particles (App. C)
# ----------------------------------------------------------------------------

def lift_profile(coarse, grid: Grid, sch: Scheme):
    """Fine node density n_k and momentum density j_k (and, with three moments, the
    second-moment density s_k) from the coarse coefficients.

    The inverse Haar transform with zero details gives the block means
    2^{-l/2} c_B.  With lift_linear, the block means sit at the block centres
    and the fine nodes take their linear interpolant (the analogue of the
    interpolation step of eq. 3.7; periodic wrap, constant beyond the end
    centres on walls); otherwise the piecewise-constant inverse Haar is used.
    """
    coarse = np.asarray(coarse, dtype=np.float64)
    nb = grid.n_cells >> sch.levels
    bs = 1 << sch.levels
    out = []
    for m in range(coarse.shape[0]):
        zeros = [np.zeros(grid.n_cells >> (i + 1)) for i in range(sch.levels)]
        const = haar_synthesis(coarse[m], zeros)  # block means on nodes 0..N-1
        means = const[::bs]
        k = np.arange(grid.n_nodes, dtype=np.float64)
        if not sch.lift_linear:
            prof = np.empty(grid.n_nodes)
            prof[: grid.n_cells] = const
            if grid.bc == WALLS:
                prof[-1] = const[-1]
            out.append(prof)
            continue
        centre = (np.arange(nb) * bs + 0.5 * (bs - 1))
        if grid.bc == PERIODIC:
            xp = np.concatenate([[centre[-1] - grid.n_cells], centre, [centre[0] + grid.n_cells]])
            fp = np.concatenate([[means[-1]], means, [means[0]]])
            out.append(np.interp(k, xp, fp))
        else:
            out.append(np.interp(k, centre, means))
    return tuple(out)


def bit_reverse32(i):
    """Reverse the 32 bits of each unsigned integer (van der Corput radical inverse in base 2)."""
    i = np.asarray(i, dtype=np.uint64)
    r = np.zeros_like(i)
    for b in range(32):
        r |= ((i >> np.uint64(b)) & np.uint64(1)) << np.uint64(31 - b)
    return r


def hammersley_b(index, shift: int):
    """Second Hammersley coordinate with a Cranley-Patterson rotation.

    b = ((bitrev32(i) + S) mod 2^32 + 1/2) / 2^32 for the global index i and the
    32-bit rotation S drawn by the caller; b lies strictly inside (0, 1).
    """
    u = (bit_reverse32(index) + np.uint64(shift)) % np.uint64(1 << 32)
    return (u.astype(np.float64) + 0.5) / 2.0 ** 32


def load_particles(n_nodes, u_nodes, grid: Grid, sch: Scheme, shift: int, t_nodes=None):
    """Quiet start from fine node profiles (App. C, particle loading).

    Every occupied cell c (some node density above n_floor) receives ppc ions
    at in-cell offsets (m + 1/2) / ppc, m = 0..ppc-1 (first Hammersley
    coordinate; positions uniform, a_i = (i + 1/2) / N_p over the whole domain).
    Velocities take the inverse CDF of a shifted Maxwellian of thermal speed
    vth at the second coordinate b_i (global index i = c ppc + m), and weights
    are the density at the particle, w = n(X) h / ppc, with n and u linearly
    interpolated between the two nodes of the cell.  With a node temperature
    profile t_nodes (three moments), the thermal speed of each ion is
    sqrt(T(X)), T linear in the cell like n and u, instead of vth.  Returns FP64
    arrays (cell, frac, v, w) in cell order; frac is the FP32 value promoted.
    """
    n_nodes = np.maximum(np.asarray(n_nodes, dtype=np.float64), 0.0)
    u_nodes = np.asarray(u_nodes, dtype=np.float64)
    nc = grid.n_cells
    right = (np.arange(nc) + 1) % nc if grid.bc == PERIODIC else np.arange(nc) + 1
    occupied = np.maximum(n_nodes[:nc], n_nodes[right]) > sch.n_floor
    cells = np.nonzero(occupied)[0]
    m = np.arange(sch.ppc)
    cell = np.repeat(cells, sch.ppc)
    mm = np.tile(m, cells.size)
    frac = ((mm + 0.5) / sch.ppc).astype(np.float32).astype(np.float64)
    idx = cell.astype(np.uint64) * np.uint64(sch.ppc) + mm.astype(np.uint64)
    b = hammersley_b(idx, shift)
    n_l, n_r = n_nodes[cell], n_nodes[right[cell]]
    u_l, u_r = u_nodes[cell], u_nodes[right[cell]]
    nx = (1.0 - frac) * n_l + frac * n_r
    ux = (1.0 - frac) * u_l + frac * u_r
    if t_nodes is None:
        sigma = sch.vth
    else:
        t_nodes = np.asarray(t_nodes, dtype=np.float64)
        sigma = np.sqrt(np.maximum((1.0 - frac) * t_nodes[cell] + frac * t_nodes[right[cell]], 0.0))
    v = ux + sigma * ndtri(b)
    w = nx * grid.h / sch.ppc
    return cell, frac, v, w


def velocity_profile(n_nodes, j_nodes, sch: Scheme):
    """Mean velocity u = j / n where the density exceeds n_floor, else 0."""
    n = np.maximum(np.asarray(n_nodes, dtype=np.float64), 0.0)
    j = np.asarray(j_nodes, dtype=np.float64)
    u = np.zeros_like(n)
    ok = n > sch.n_floor
    u[ok] = j[ok] / n[ok]
    return u


def temperature_profile(n_nodes, j_nodes, s_nodes, sch: Scheme):
    """Ion temperature T = s / n - u^2 (the pressure over the density, P = s - n u^2)
    where the density exceeds n_floor, clipped at 0; else 0."""
    n = np.maximum(np.asarray(n_nodes, dtype=np.float64), 0.0)
    j = np.asarray(j_nodes, dtype=np.float64)
    s = np.asarray(s_nodes, dtype=np.float64)
    t = np.zeros_like(n)
    ok = n > sch.n_floor
    u = j[ok] / n[ok]
    t[ok] = np.maximum(s[ok] / n[ok] - u * u, 0.0)
    return t


def block_correct(cell, v, w, coarse, grid: Grid, sch: Scheme):
    """Per-block mass and momentum (and second-moment) correction of lifted particles.

    Block B holds the particles of cells c with c >> l = B.  Its weights are
    rescaled so that their sum is the block mass M = h 2^{l/2} max(c^n_B, 0), then
    its velocities are shifted so that sum w v is the block momentum
    J = h 2^{l/2} c^j_B (the "Maxwellian-corrected" resampling; the negative values
    of the remark in Sec. 3.3 are clipped).  With three coarse moments the
    velocities are also stretched about the block's mean velocity so that
    sum w v^2 is the block's second moment S = h 2^{l/2} c^s_B: with the rescaled
    weights, mean velocity u_g and spread G = sum w (v - u_g)^2 of the loaded
    ions, v <- J / M + a (v - u_g), a = sqrt(max(S - J^2 / M, 0) / G).  Blocks
    without particles or mass are left unchanged.
    """
    coarse = np.asarray(coarse, dtype=np.float64)
    nb = grid.n_cells >> sch.levels
    scale = grid.h * 2.0 ** (sch.levels / 2.0)
    blk = np.asarray(cell) >> sch.levels
    w = np.array(w, dtype=np.float64)
    v = np.array(v, dtype=np.float64)
    mass_t = np.maximum(coarse[0], 0.0) * scale
    mom_t = coarse[1] * scale
    s = np.bincount(blk, weights=w, minlength=nb)
    ratio = np.ones(nb)
    ok = s > 0.0
    ratio[ok] = mass_t[ok] / s[ok]
    w = w * ratio[blk]
    p = np.bincount(blk, weights=w * v, minlength=nb)
    okm = mass_t > 0.0
    if coarse.shape[0] < 3:
        dv = np.zeros(nb)
        dv[okm] = (mom_t[okm] - p[okm]) / mass_t[okm]
        return v + dv[blk], w
    second_t = coarse[2] * scale
    u_g = np.zeros(nb)
    u_t = np.zeros(nb)
    u_g[okm] = p[okm] / mass_t[okm]
    u_t[okm] = mom_t[okm] / mass_t[okm]
    spread = np.bincount(blk, weights=w * (v - u_g[blk]) ** 2, minlength=nb)
    a = np.ones(nb)
    oks = okm & (spread > 0.0)
    a[oks] = np.sqrt(np.maximum(second_t[oks] - mom_t[oks] ** 2 / mass_t[oks], 0.0) / spread[oks])
    moved = okm[blk]
    v = np.where(moved, u_t[blk] + a[blk] * (v - u_g[blk]), v)
    return v, w


def lift(coarse, grid: Grid, sch: Scheme, shift: int, correct=True):
    """Lifting operator: coarse coefficients -> quiet-start particles (Sec. 3.3, App. C).

    With three coarse moments the loaded Maxwellian takes the local temperature
    of the profiles (EFREE, Sec. 3.2) instead of the fixed vth."""
    prof = lift_profile(coarse, grid, sch)
    u_f = velocity_profile(prof[0], prof[1], sch)
    t_f = temperature_profile(*prof, sch) if len(prof) > 2 else None
    cell, frac, v, w = load_particles(prof[0], u_f, grid, sch, shift, t_f)
    if correct:
        v, w = block_correct(cell, v, w, coarse, grid, sch)
    return cell, frac, v, w


# ----------------------------------------------------------------------------
# The projective cycle (Sec. 3.1 with eq. 3.17, App. B restriction)
# ----------------------------------------------------------------------------

def pic_burst(x, v, w, grid: Grid, sch: Scheme, steps=None, alive=None, phi0=None):
    """Fine burst with restriction after every step: p = 0..N_e snapshots.

    x, v: positions and integer-time velocities after lifting.  The field E_n
    at the start of the burst is stored (App. B, step 1).  At fine step p the
    time-centred velocity v^p = v^{p-1/2} + dt/2 E^p(X^p) is restricted with
    tau = Delta t - p dt; then the leapfrog step advances to p + 1.
    Returns (snapshots (N_e+1, 2, N_c), x, v_half, alive, phi).
    """
    ne = sch.burst_steps if steps is None else steps
    x = np.array(x, dtype=np.float64)
    w = np.array(w, dtype=np.float64)
    alive = np.ones(x.shape, bool) if alive is None else np.array(alive)
    _, phi, e = pic.field_from_particles(x, w, alive, grid, phi0)
    e_n = e.copy()
    vh = np.array(v, dtype=np.float64)
    vh[alive] -= 0.5 * grid.dt * pic.gather(e, x[alive], grid)
    snaps = []
    for p in range(ne + 1):
        ep = pic.gather(e, x[alive], grid)
        vp = vh[alive] + 0.5 * grid.dt * ep
        tau = sch.macro_dt - p * grid.dt
        en_x = pic.gather(e_n, x[alive], grid)
        snaps.append(restrict_snapshot(x[alive], vp, en_x, w[alive], tau, grid,
                                       sch.levels, sch.coevolving, sch.moments))
        if p < ne:
            x, vh, alive = pic.leapfrog_step(x, vh, w, alive, e, grid)
            _, phi, e = pic.field_from_particles(x, w, alive, grid, phi)
    return np.array(snaps), x, vh, alive, phi


def particles_to_x(cell, frac, grid: Grid):
    return (np.asarray(cell, dtype=np.float64) + np.asarray(frac, dtype=np.float64)) * grid.h


def macro_step(coarse, grid: Grid, sch: Scheme, shift: int, phi0=None):
    """One EFPI macro step: lift, burst with restriction, least squares, projection."""
    cell, frac, v, w = lift(coarse, grid, sch, shift)
    x = particles_to_x(cell, frac, grid)
    snaps, _, _, _, phi = pic_burst(x, v, w, grid, sch, phi0=phi0)
    return project(snaps, grid.dt, sch.macro_dt), snaps, phi


def restrict_state(x, v, w, alive, grid: Grid, sch: Scheme):
    """Plain restriction (tau = 0) of a particle state: the coarse variables at that time."""
    z = np.zeros(int(np.sum(alive)))
    return restrict_snapshot(x[alive], v[alive], z, w[alive], 0.0, grid, sch.levels, False,
                             sch.moments)


def ensemble_mean(coarse_list):
    """Arithmetic mean of the coarse arrays of replicas sharing a grid, in replica order."""
    acc = np.zeros_like(np.asarray(coarse_list[0], dtype=np.float64))
    for c in coarse_list:
        acc = acc + np.asarray(c, dtype=np.float64)
    return acc / len(coarse_list)
