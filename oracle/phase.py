"""Oracle of the phase-space (wavelet) coarse variables, FP64.  TEST
INFRASTRUCTURE ONLY (see package header).

The wavelet-based scheme of Sec. 3.3 represents the ion distribution f(x, v) on
a fine phase-space grid: nodes x_k = k h (piecewise linear in x, the CIC hat)
and n_vf = 2^{J_f} velocity bins of width dv over [V_min, V_max) (piecewise
constant in v).  Coarsening applies l levels of the full-weighting restriction
(eq. 3.8) in x, then the periodized discrete wavelet transform of every
velocity column down to J_c (App. A), keeping the 2^{J_c} scaling coefficients.
Lifting inverts the transform with zero details, interpolates in x (eq. 3.7),
builds per fine node the conditional CDF in v, repairs it (App. C) and loads
ions by the quiet start with the inverse of the repaired CDF.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.optimize import least_squares

from . import efpi, pic
from .pic import Grid, PERIODIC


@dataclass
class PhaseScheme:
    """Phase-space coarse representation of one replica."""

    levels: int = 4          # l: full-weighting levels in x
    v_min: float = -2.0      # velocity window [v_min, v_max)
    v_max: float = 2.0
    jf: int = 8              # n_vf = 2^jf fine velocity bins
    jc: int = 5              # n_vc = 2^jc coarse scaling coefficients per x node
    burst_steps: int = 20
    macro_dt: float = 7.5
    coevolving: bool = True
    ppc: int = 100
    n_floor: float = 1e-6

    @property
    def n_vf(self) -> int:
        return 1 << self.jf

    @property
    def n_vc(self) -> int:
        return 1 << self.jc

    @property
    def dv(self) -> float:
        return (self.v_max - self.v_min) / self.n_vf


# ----------------------------------------------------------------------------
# The order-4 Coiflet filter (App. A)
# ----------------------------------------------------------------------------

COIFLET_TAPS = 12
COIFLET_ORIGIN = 4   # tap index of the origin of the support [-4, 7]


def coiflet_conditions(h):
    """Residuals of the conditions that define the filter (App. A): sum h = sqrt 2,
    orthonormality of its even shifts, four vanishing moments of the wavelet
    (high-pass g_k = (-1)^k h_{L-1-k}) and vanishing moments 1..3 of the scaling
    function about the origin of its support.  The paper states the scaling
    moments about y = 0; for taps indexed 0..11 that origin is tap 4 (support
    [-4, 7]).  Through the two-scale relation, these discrete moments of the taps
    vanish exactly when the continuous moments of phi and psi do."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    k = np.arange(n, dtype=np.float64)
    r = [h.sum() - np.sqrt(2.0), np.dot(h, h) - 1.0]
    for m in range(1, n // 2):
        r.append(np.dot(h[: n - 2 * m], h[2 * m:]))
    g = ((-1.0) ** k) * h[::-1]
    for p in range(4):
        r.append(np.sum(g * k ** p))
    for p in (1, 2, 3):
        r.append(np.sum(h * (k - COIFLET_ORIGIN) ** p))
    return np.array(r)


def scaling_function(h, levels: int):
    """The scaling function at the dyadic points i 2^-levels of its support [0, L-1]
    (taps indexed from 0), by the cascade: its values at the integers are the
    eigenvector of eigenvalue 1 of the refinement matrix sqrt 2 h_{2n-m}, summing
    to 1, and each level follows from phi(y) = sqrt 2 sum_k h_k phi(2y - k)."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    a = np.zeros((n, n))
    for i in range(n):
        for m in range(n):
            if 0 <= 2 * i - m < n:
                a[i, m] = np.sqrt(2.0) * h[2 * i - m]
    w, vec = np.linalg.eig(a)
    phi = np.real(vec[:, np.argmin(np.abs(w - 1.0))])
    phi = phi / phi.sum()
    for j in range(levels):
        step = 1 << j
        size = (n - 1) * 2 * step + 1
        nxt = np.zeros(size)
        for k in range(n):
            src = np.arange(size) - k * step
            ok = (src >= 0) & (src < phi.size)
            nxt[ok] += np.sqrt(2.0) * h[k] * phi[src[ok]]
        phi = nxt
    return phi


def coiflet_filter(starts: int = 60) -> np.ndarray:
    """The 12-tap order-4 Coiflet.  coiflet_conditions has several isolated
    solutions; they are found by least squares from seeded starting points, and
    the one whose scaling function (cascade, 2^-10 grid) is most nearly symmetric
    about the support origin is returned (the paper picks this family for its
    regularity and symmetry)."""
    rng = np.random.default_rng(0)
    sols = []
    for _ in range(starts):
        sol = least_squares(coiflet_conditions, rng.normal(0.0, 0.3, COIFLET_TAPS),
                            xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=20000)
        if np.max(np.abs(coiflet_conditions(sol.x))) < 1e-12 and \
                not any(np.max(np.abs(sol.x - s)) < 1e-8 for s in sols):
            sols.append(sol.x)
    if not sols:
        raise RuntimeError("no Coiflet filter found")
    levels = 10
    o = COIFLET_ORIGIN << levels

    def asymmetry(h):
        phi = scaling_function(h, levels)
        right = phi[o:]
        left = np.zeros(right.size)
        left[: o + 1] = phi[o::-1]
        return np.sum((right - left) ** 2) * 2.0 ** -levels

    return min(sols, key=asymmetry)


def highpass(h):
    k = np.arange(h.size)
    return ((-1.0) ** k) * np.asarray(h)[::-1]


# ----------------------------------------------------------------------------
# Periodized discrete wavelet transform (App. A)
# ----------------------------------------------------------------------------

def dwt_level(x, h):
    """One periodized analysis level along the last axis:
    a_k = sum_m h_m x_{(2k+m) mod N}, d_k = sum_m g_m x_{(2k+m) mod N}."""
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[-1]
    idx = (2 * np.arange(n // 2)[:, None] + np.arange(len(h))[None, :]) % n
    return x[..., idx] @ np.asarray(h), x[..., idx] @ highpass(h)


def idwt_level(a, d, h):
    """Inverse of dwt_level along the last axis: coefficient k spreads
    h_m a_k + g_m d_k onto sample (2k + m) mod N (d = None: zero details)."""
    a = np.asarray(a, dtype=np.float64)
    half = a.shape[-1]
    n = 2 * half
    g = highpass(h)
    x = np.zeros(a.shape[:-1] + (n,))
    for m in range(len(h)):
        tgt = (2 * np.arange(half) + m) % n
        contrib = h[m] * a if d is None else h[m] * a + g[m] * np.asarray(d)
        np.add.at(x, (..., tgt), contrib) if x.ndim > 1 else np.add.at(x, tgt, contrib)
    return x


def scaling_coefficients(col, h, levels: int):
    """Scaling coefficients `levels` levels below the columns (last axis; details dropped)."""
    a = np.asarray(col, dtype=np.float64)
    for _ in range(levels):
        a, _ = dwt_level(a, h)
    return a


def from_scaling_coefficients(a, h, levels: int):
    """Column `levels` levels above the scaling coefficients a, with zero details."""
    x = np.asarray(a, dtype=np.float64)
    for _ in range(levels):
        x = idwt_level(x, None, h)
    return x


# ----------------------------------------------------------------------------
# Spatial restriction and interpolation (eqs. 3.7-3.8), periodic
# ----------------------------------------------------------------------------

def full_weighting(f):
    """One level of eq. 3.8 along axis 0: coarse k = (f_{2k-1} + 2 f_{2k} + f_{2k+1}) / 4."""
    f = np.asarray(f, dtype=np.float64)
    even = f[0::2]
    odd = f[1::2]
    return 0.25 * (np.roll(odd, 1, axis=0) + 2.0 * even + odd)


def midpoint_interpolation(f):
    """One level of eq. 3.7 along axis 0: fine 2k = f_k, fine 2k + 1 = (f_k + f_{k+1}) / 2."""
    f = np.asarray(f, dtype=np.float64)
    out = np.empty((2 * f.shape[0],) + f.shape[1:])
    out[0::2] = f
    out[1::2] = 0.5 * (f + np.roll(f, -1, axis=0))
    return out


# ----------------------------------------------------------------------------
# Restriction: particles -> phase-space histogram -> coarse coefficients
# ----------------------------------------------------------------------------

def phase_histogram(x, v, w, grid: Grid, ps: PhaseScheme):
    """Fine histogram f[k_x][k_v] of the particles (eq. for the fine representation
    in Sec. 3.3): CIC weights in x on the nodes, nearest bin in v, divided by h dv
    (a phase-space density).  Particles outside [v_min, v_max) are not counted."""
    assert grid.bc == PERIODIC
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    kv = np.floor((v - ps.v_min) / ps.dv).astype(np.int64)
    ok = (kv >= 0) & (kv < ps.n_vf)
    c, th = pic.cic_nodes(x[ok], grid)
    c = c % grid.n_cells
    r = (c + 1) % grid.n_cells
    f = np.zeros((grid.n_cells, ps.n_vf))
    np.add.at(f, (c, kv[ok]), (1.0 - th) * w[ok])
    np.add.at(f, (r, kv[ok]), th * w[ok])
    return f / (grid.h * ps.dv)


def restricted_histogram_fx(cell, frac, v, w, n_cells: int, ps: PhaseScheme):
    """The histogram after l full-weighting levels, in exact integer arithmetic
    (the form the GPU accumulates): the charge q = rint(w 2^40) of each ion is
    split as in the deposit, q_R = rint(theta q), q_L = q - q_R, and fine node
    i = 2^l K + d adds (2^l - d) and d times its share to coarse nodes K and
    K + 1 (the composed weights of eq. 3.8, with denominator 4^l).  Ions in cell
    c at offset theta (FP32), velocities v; bin floor((v - v_min) / dv).
    Returns int64 H[n_cells >> l][n_vf]; H 2^-40 / (4^l h dv) equals l levels of
    full_weighting applied to phase_histogram."""
    cell = np.asarray(cell).astype(np.int64)
    frac = np.asarray(frac, dtype=np.float32).astype(np.float64)
    v = np.asarray(v, dtype=np.float64)
    w = np.asarray(w, dtype=np.float32).astype(np.float64)
    kv = np.floor((v - ps.v_min) / ps.dv).astype(np.int64)
    ok = (cell >= 0) & (kv >= 0) & (kv < ps.n_vf)
    cell, frac, kv, w = cell[ok], frac[ok], kv[ok], w[ok]
    q = np.rint(w * pic.FX_SCALE).astype(np.int64)
    qr = np.rint(frac * q.astype(np.float64)).astype(np.int64)
    ql = q - qr
    nxc = n_cells >> ps.levels
    span = 1 << ps.levels
    H = np.zeros((nxc, ps.n_vf), dtype=np.int64)
    for node, share in ((cell, ql), ((cell + 1) % n_cells, qr)):
        K = node >> ps.levels
        d = node & (span - 1)
        np.add.at(H, (K, kv), share * (span - d))
        np.add.at(H, ((K + 1) % nxc, kv), share * d)
    return H


def coarse_from_histogram_fx(H, ps: PhaseScheme, h_grid: float, h):
    """Coarse coefficients from restricted_histogram_fx: the phase-space density
    H 2^-40 / (4^l h dv), scaled to App. A's finest coefficients, then the wavelet
    transform of each column down to J_c."""
    dens = np.asarray(H, dtype=np.float64) / pic.FX_SCALE / (4.0 ** ps.levels * h_grid * ps.dv)
    scale = 2.0 ** (-ps.jf / 2.0) * (ps.v_max - ps.v_min)
    return scaling_coefficients(scale * dens, h, ps.jf - ps.jc)


def coarsen(f, ps: PhaseScheme, h):
    """l levels of full weighting in x, then per coarse x node the scaling
    coefficients at J_c of the column, whose finest-level coefficients are
    2^{-J_f/2} times the histogram in the velocity rescaled to [0, 1) (App. A)."""
    g = np.asarray(f, dtype=np.float64)
    for _ in range(ps.levels):
        g = full_weighting(g)
    scale = 2.0 ** (-ps.jf / 2.0) * (ps.v_max - ps.v_min)
    return scaling_coefficients(scale * g, h, ps.jf - ps.jc)


def restrict_phase(x, v, e_n_at_x, w, tau, grid: Grid, ps: PhaseScheme, h):
    """Coarse coefficients [n_xc][n_vc] of one snapshot along the co-evolving frame
    (App. B): the histogram of (X + tau v, v + tau E_n(X)), coarsened."""
    xt = np.mod(np.asarray(x) + tau * np.asarray(v), grid.length)
    vt = np.asarray(v) + tau * np.asarray(e_n_at_x)
    return coarsen(phase_histogram(xt, vt, w, grid, ps), ps, h)


# ----------------------------------------------------------------------------
# Lifting: coarse coefficients -> fine histogram -> repaired CDFs -> particles
# ----------------------------------------------------------------------------

def refine(coarse, ps: PhaseScheme, h):
    """Inverse of coarsen with zero details: columns back to J_f, then l levels of
    midpoint interpolation in x; returns the fine histogram f[k_x][k_v]."""
    scale = 2.0 ** (ps.jf / 2.0) / (ps.v_max - ps.v_min)
    g = scale * from_scaling_coefficients(coarse, h, ps.jf - ps.jc)
    for _ in range(ps.levels):
        g = midpoint_interpolation(g)
    return g


def _seqsum(a):
    """Sum in index order (the repair's decisions compare such sums, so the order
    is part of the definition here)."""
    a = np.asarray(a, dtype=np.float64)
    return float(np.cumsum(a)[-1]) if a.size else 0.0


def column_cdf(col, dv):
    """Node density n = (sum f) dv and the conditional CDF at the bin edges,
    F[k] = ((sum_{j<k} f_j) dv) / n (F[0] = 0, F[n_vf] = 1); sums in index order."""
    col = np.asarray(col, dtype=np.float64)
    run = np.cumsum(col)
    n = float(run[-1]) * dv
    F = np.concatenate([[0.0], (run * dv) / n])
    F[-1] = 1.0
    return n, F


def _edge_low(F):
    """Edge reconstruction of App. C for entries below 0 (momentum-conserving
    ramp from 0 up to the first index past the last negative entry)."""
    F = F.copy()
    nf = F.size - 1
    neg = np.nonzero(F < 0.0)[0]
    if neg.size == 0:
        return F
    k0 = int(neg[-1])
    km, kp = k0 - 1, k0 + 1
    while True:
        span = kp - km
        dF = 2.0 * _seqsum(F[1:kp]) / (span * (span - 1))
        if 0.0 <= (span - 1) * dF <= F[kp] or kp >= nf:
            break
        if km > 0:
            km -= 1
        else:
            kp += 1
            km = k0 - 1
    F[:max(km, 0)] = 0.0
    for k in range(max(km, 0), kp):
        F[k] = (k - km) * dF
    return F


def _edges(F):
    """Both edges: entries below 0 as above, entries above 1 by the same rule on
    the reflected array 1 - F[n - k]."""
    F = _edge_low(F)
    G = _edge_low(1.0 - F[::-1])
    return 1.0 - G[::-1]


def _interior_forward(F):
    """Interior reconstruction of App. C from the lower indexes: each decrease is
    replaced by a momentum-conserving ramp between k_- and k_+.  The acceptance
    test is read as the ramp's last value F[k_-] + (k_+ - k_- - 1) dF not
    exceeding F[k_+] (monotone at k_+; the printed test omits F[k_-])."""
    F = F.copy()
    nf = F.size - 1
    k0 = 0
    while True:
        drops = np.nonzero(F[k0:-1] > F[k0 + 1:])[0]
        if drops.size == 0:
            return F
        k0 = k0 + int(drops[0])
        up = np.nonzero(F[k0 + 1:] >= F[k0])[0]
        k1 = k0 + 1 + int(up[0]) if up.size else nf
        kp = k0 + 1 + int(np.argmin(F[k0 + 1:k1 + 1]))
        below = np.nonzero(F[:k0] <= F[kp])[0]
        km = int(below[-1]) if below.size else 0
        while True:
            span = kp - km
            dF = 2.0 / (span - 1) * (_seqsum(F[km:kp]) / span - F[km])
            if 0.0 <= (span - 1) * dF and F[km] + (span - 1) * dF <= F[kp]:
                break
            if kp >= nf:
                # no momentum-conserving ramp fits below F[n] (the pathological case
                # the paper sets aside): join F[k-] to F[n] by a straight line
                dF = (F[nf] - F[km]) / (nf - km)
                kp = nf
                break
            kp += 1
        for k in range(km + 1, kp):
            F[k] = F[km] + (k - km) * dF
        k0 = kp  # F is monotone on [0, k+]


def repair_cdf(F):
    """The reconstruction RF of App. C: edges, then the interior correction from
    the lower indexes (F+) and from the upper ones (F-, on the reflected array),
    averaged."""
    F = _edges(np.asarray(F, dtype=np.float64))
    fp = _interior_forward(F)
    fm = 1.0 - _interior_forward(1.0 - F[::-1])[::-1]
    return 0.5 * (fp + fm)


def inverse_cdf(RF, b, ps: PhaseScheme):
    """v with RF(v) = b: the bin k with RF[k] <= b < RF[k+1] (lookup), linear in it."""
    RF = np.asarray(RF)
    b = np.asarray(b, dtype=np.float64)
    k = np.searchsorted(RF, b, side="right") - 1
    k = np.clip(k, 0, RF.size - 2)
    lo, hi = RF[k], RF[k + 1]
    t = np.where(hi > lo, (b - lo) / np.where(hi > lo, hi - lo, 1.0), 0.5)
    return ps.v_min + (k + t) * ps.dv


def lift_phase(coarse, grid: Grid, ps: PhaseScheme, h, shift: int):
    """Ions from the coarse coefficients (App. C particle loading): fine histogram
    by refine, per node density and repaired CDF, then per occupied cell ppc ions
    at offsets (m + 1/2)/ppc with velocity the inverse CDFs of the two nodes at the
    Hammersley b (rotation `shift`) interpolated linearly in x, and weight
    n(X) h / ppc.  Returns (cell, frac, v, w) in cell order."""
    f = refine(coarse, ps, h)
    nc = grid.n_cells
    dens = np.zeros(nc)
    cdfs = []
    for k in range(nc):
        n, F = column_cdf(f[k], ps.dv)
        dens[k] = n
        cdfs.append(repair_cdf(F) if n > ps.n_floor else None)
    right = (np.arange(nc) + 1) % nc
    occupied = np.maximum(dens, dens[right]) > ps.n_floor
    cells = np.nonzero(occupied)[0]
    m = np.arange(ps.ppc)
    cell = np.repeat(cells, ps.ppc)
    mm = np.tile(m, cells.size)
    frac = ((mm + 0.5) / ps.ppc).astype(np.float32).astype(np.float64)
    idx = cell.astype(np.uint64) * np.uint64(ps.ppc) + mm.astype(np.uint64)
    b = efpi.hammersley_b(idx, shift)
    v = np.zeros(cell.size)
    for c in cells:
        sel = cell == c
        vl = inverse_cdf(cdfs[c], b[sel], ps) if cdfs[c] is not None else 0.0
        vr = inverse_cdf(cdfs[right[c]], b[sel], ps) if cdfs[right[c]] is not None else vl
        if cdfs[c] is None:
            vl = vr
        th = frac[sel]
        v[sel] = (1.0 - th) * vl + th * vr
    nx = (1.0 - frac) * np.maximum(dens[cell], 0.0) + frac * np.maximum(dens[right[cell]], 0.0)
    w = nx * grid.h / ps.ppc
    return cell, frac, v, w


# ----------------------------------------------------------------------------
# The macro step on phase-space coefficients (Sec. 3.1 with eqs. 3.17-3.18)
# ----------------------------------------------------------------------------

def phase_burst(x, v, w, grid: Grid, ps: PhaseScheme, h, phi0=None):
    """Fine burst (Boltzmann electrons, oracle.pic) with the phase-space
    restriction after every step along the co-evolving frame; returns the
    snapshots [N_e + 1][n_xc][n_vc]."""
    x = np.array(x, dtype=np.float64)
    w = np.array(w, dtype=np.float64)
    alive = np.ones(x.shape, bool)
    _, phi, e = pic.field_from_particles(x, w, alive, grid, phi0)
    e_n = e.copy()
    vh = np.array(v, dtype=np.float64) - 0.5 * grid.dt * pic.gather(e, x, grid)
    snaps = []
    for p in range(ps.burst_steps + 1):
        vp = vh + 0.5 * grid.dt * pic.gather(e, x, grid)
        tau = (ps.macro_dt - p * grid.dt) if ps.coevolving else 0.0
        snaps.append(restrict_phase(x, vp, pic.gather(e_n, x, grid), w, tau, grid, ps, h))
        if p < ps.burst_steps:
            x, vh, alive = pic.leapfrog_step(x, vh, w, alive, e, grid)
            _, phi, e = pic.field_from_particles(x, w, alive, grid, phi)
    return np.array(snaps)


def phase_macro_step(coarse, grid: Grid, ps: PhaseScheme, h, shift: int):
    """Lift, burst with phase-space restriction, least squares and projection."""
    cell, frac, v, w = lift_phase(coarse, grid, ps, h, shift)
    x = efpi.particles_to_x(cell, frac, grid)
    snaps = phase_burst(x, v, w, grid, ps, h)
    return efpi.project(snaps, grid.dt, ps.macro_dt), snaps
