"""Pins of the oracle's coarse representation, projection and lifting.

Checks use closed forms (block sums, Parseval, least squares by a library
routine, exact free streaming), invariants stated by the paper (charge
conservation of the projection, Sec. 3.3 remark) and statistical properties
of the quiet start (App. C).
"""
import numpy as np
import pytest
from scipy.special import ndtr

from oracle import efpi, pic, metrics
from oracle.pic import Grid, PERIODIC, WALLS, NOFIELD
import synth


# ------------------------------------------------------------------ Haar ----

def test_haar_block_sum_closed_form_and_parseval():
    g = np.random.default_rng(0)
    f = g.standard_normal(256)
    s, d = efpi.haar_analysis(f, 4)
    assert np.allclose(s, f.reshape(16, 16).sum(axis=1) / 4.0, atol=1e-13)
    energy = np.sum(s ** 2) + sum(np.sum(x ** 2) for x in d)
    assert energy == pytest.approx(np.sum(f ** 2), rel=1e-13)
    assert np.allclose(efpi.haar_synthesis(s, d), f, atol=1e-13)


def test_haar_constant():
    s, d = efpi.haar_analysis(np.full(64, 3.0), 3)
    assert np.allclose(s, 3.0 * 2 ** 1.5) and all(np.allclose(x, 0.0) for x in d)


def test_restriction_total_charge():
    g = Grid(128, 128.0)
    cell, frac, v, w = synth.random_particles(3000, 128, seed=4)
    x = efpi.particles_to_x(cell, frac.astype(float), g)
    c = efpi.restrict_snapshot(x, v.astype(float), np.zeros(x.size), w.astype(float), 0.0, g, 3, False)
    assert c[0].sum() * 2 ** 1.5 * g.h == pytest.approx(w.astype(float).sum(), rel=1e-13)
    assert c[1].sum() * 2 ** 1.5 * g.h == pytest.approx(np.sum(w.astype(float) * v), rel=1e-12)


def test_restriction_walls_fold_and_exclusion():
    g = Grid(16, 16.0, WALLS)
    # A particle at 15.5 shares half to node 16, which joins the last block.
    c = efpi.restrict_snapshot(np.array([15.5]), np.array([0.0]), np.zeros(1), np.array([1.0]),
                               0.0, g, 2, False)
    assert c[0][-1] * 2.0 == pytest.approx(1.0) and np.allclose(c[0][:-1], 0.0)
    # moved beyond the wall by the characteristic: excluded from the snapshot
    c = efpi.restrict_snapshot(np.array([15.5]), np.array([1.0]), np.zeros(1), np.array([1.0]),
                               1.0, g, 2, True)
    assert np.allclose(c, 0.0)


# ------------------------------------------------------- least squares ------

@pytest.mark.parametrize("ne", [1, 2, 6, 10, 20])
def test_ls_slope_equals_polyfit(ne):
    g = np.random.default_rng(ne)
    dt = 0.1
    snaps = g.standard_normal((ne + 1, 2, 8))
    slope = efpi.ls_slope(snaps, dt)
    t = np.arange(ne + 1) * dt
    ref = np.polyfit(t, snaps.reshape(ne + 1, -1), 1)[0].reshape(2, 8)
    assert np.allclose(slope, ref, atol=1e-10)


def test_ls_exact_on_linear_data_and_shift_invariant():
    dt = 0.1
    base = np.random.default_rng(1).standard_normal((2, 8))
    rate = np.random.default_rng(2).standard_normal((2, 8))
    snaps = np.array([base + rate * p * dt for p in range(21)])
    assert np.allclose(efpi.ls_slope(snaps, dt), rate, atol=1e-12)
    assert np.allclose(efpi.ls_slope(snaps + 5.0, dt), rate, atol=1e-11)
    # projection of exactly linear data is exact
    nxt = efpi.project(snaps, dt, 20.0)
    assert np.allclose(nxt, base + rate * 20.0, atol=1e-10)


def test_projection_conserves_charge():
    # Remark of Sec. 3.3: equal totals in every snapshot -> the slope sums to zero.
    g = np.random.default_rng(3)
    snaps = g.standard_normal((21, 2, 16))
    snaps -= snaps.sum(axis=2, keepdims=True) / 16
    snaps += 1.0
    slope = efpi.ls_slope(snaps, 0.1)
    assert abs(slope[0].sum()) < 1e-12
    assert efpi.project(snaps, 0.1, 20.0)[0].sum() == pytest.approx(16.0, rel=1e-13)


# ------------------------------------------ second-order projective step ---

def _quadratic_bursts(ne, dt, gap, macro_dt, seed):
    """Snapshots of c(t) = a + b t + q t^2 for the previous burst (starting at
    -gap) and the current one (starting at 0), and c at t = macro_dt."""
    g = np.random.default_rng(seed)
    a, b, q = (g.standard_normal((2, 8)) for _ in range(3))
    c = lambda t: a + b * t + q * t * t
    prev = np.array([c(-gap + p * dt) for p in range(ne + 1)])
    cur = np.array([c(p * dt) for p in range(ne + 1)])
    return prev, cur, c(macro_dt), q


@pytest.mark.parametrize("ne,gap,macro_dt", [(20, 7.5, 7.5), (10, 5.0, 6.0), (6, 8.0, 4.0)])
def test_project2_exact_on_quadratic_trajectories(ne, gap, macro_dt):
    # For a quadratic trajectory the LS slope of a burst is the derivative at its
    # centre, the derivative is linear, and its value at the middle of the leap
    # integrates it exactly: the second-order step lands on c(Delta t); the
    # forward-Euler step misses by the curvature term.
    dt = 0.1
    prev, cur, exact, q = _quadratic_bursts(ne, dt, gap, macro_dt, ne)
    f_prev = efpi.ls_slope(prev, dt)
    f, euler, second = efpi.project2(cur, dt, macro_dt, f_prev, gap)
    assert np.allclose(f, efpi.ls_slope(cur, dt))
    assert np.max(np.abs(second - exact)) < 1e-10 * np.max(np.abs(exact))
    leap = macro_dt - ne * dt
    # Euler: c(t_e) + leap c'(centre) differs from c(Delta t) by q leap Delta t
    assert np.allclose(exact - euler, q * leap * macro_dt, atol=1e-9)


def test_project2_reduces_to_euler():
    g = np.random.default_rng(5)
    snaps = g.standard_normal((21, 2, 16))
    f, euler, second = efpi.project2(snaps, 0.1, 7.5)
    assert np.array_equal(euler, second)
    assert np.allclose(euler, efpi.project(snaps, 0.1, 7.5), rtol=0, atol=1e-14)
    _, euler2, second2 = efpi.project2(snaps, 0.1, 7.5, f, 7.5)
    assert np.array_equal(euler2, second2)


def test_project2_conserves_charge():
    # Equal totals in every snapshot of both bursts -> both slopes sum to zero,
    # so the second-order step keeps the total charge (as eq. 3.17 does).
    g = np.random.default_rng(6)
    def burst():
        sn = g.standard_normal((21, 2, 16))
        sn -= sn.sum(axis=2, keepdims=True) / 16
        return sn + 1.0
    f_prev = efpi.ls_slope(burst(), 0.1)
    _, _, second = efpi.project2(burst(), 0.1, 7.5, f_prev, 6.0)
    assert second[0].sum() == pytest.approx(16.0, rel=1e-13)


def test_step_rule_meets_tolerance_under_its_error_model():
    # If the Euler-step error is C Delta t^2, the next step's error is safety^2 tol
    # (inside the factor-2 and [dt_min, dt_max] limits), and the rule is monotone.
    tol, safety = 1e-3, 0.9
    for C, dt in ((2e-5, 6.0), (1e-4, 4.0), (4e-5, 5.0)):
        err = C * dt * dt
        nxt = efpi.next_macro_dt(dt, err, tol, 0.1, 100.0, safety)
        if 0.5 * dt < nxt < 2.0 * dt:
            assert C * nxt * nxt == pytest.approx(safety ** 2 * tol, rel=1e-12)
    steps = [efpi.next_macro_dt(5.0, e, tol, 2.0, 7.5) for e in (0.0, 1e-5, 1e-4, 1e-3, 1e-2, 1.0)]
    assert steps == sorted(steps, reverse=True)
    assert steps[0] == 7.5 and steps[-1] == 2.5
    assert efpi.next_macro_dt(2.1, 1.0, tol, 2.0, 7.5) == 2.0


# ------------------------------------------------------ co-evolving frame ---

def test_coevolving_frame_exact_in_free_streaming():
    # E = 0: X~ = X^0 + Delta t V for every p (App. B, eq. B.4), so all snapshots
    # agree, the slope vanishes and the projection equals the restriction of the
    # exactly free-streamed state at t + Delta t.
    g = Grid(64, 64.0, closure=NOFIELD)
    sch = efpi.Scheme(levels=2, burst_steps=6, macro_dt=3.0, ppc=32)
    nn, uu = synth.iaw_profile(64, 64.0)
    cell, frac, v, w = efpi.load_particles(nn, uu, g, sch, synth.lift_shift(5))
    x = efpi.particles_to_x(cell, frac, g)
    snaps, *_ = efpi.pic_burst(x, v, w, g, sch)
    assert np.max(np.abs(snaps - snaps[0])) < 1e-10
    assert np.max(np.abs(efpi.ls_slope(snaps, g.dt))) < 1e-8
    xf = np.mod(x + sch.macro_dt * v, g.length)
    ref = efpi.restrict_snapshot(xf, v, np.zeros_like(v), w, 0.0, g, 2, False)
    nxt = efpi.project(snaps, g.dt, sch.macro_dt)
    assert np.max(np.abs(nxt - ref)) < 1e-8


def test_plain_restriction_changes_under_streaming():
    g = Grid(64, 64.0, closure=NOFIELD)
    sch = efpi.Scheme(levels=2, burst_steps=6, macro_dt=3.0, ppc=32, coevolving=False)
    nn, uu = synth.iaw_profile(64, 64.0)
    cell, frac, v, w = efpi.load_particles(nn, uu, g, sch, synth.lift_shift(5))
    snaps, *_ = efpi.pic_burst(efpi.particles_to_x(cell, frac, g), v, w, g, sch)
    assert np.max(np.abs(snaps - snaps[0])) > 1e-4


# ------------------------------------------------------------------ lift ----

def test_hammersley_radical_inverse_definition():
    idx = np.array([0, 1, 2, 3, 6, 12345, 2 ** 31 + 7], dtype=np.uint64)
    # van der Corput by its digit expansion: sum of bit_b 2^{-(b+1)}
    vdc = np.array([sum(((int(i) >> b) & 1) * 2.0 ** -(b + 1) for b in range(32)) for i in idx])
    b = efpi.hammersley_b(idx, 0)
    assert np.allclose(b, vdc + 2.0 ** -33, atol=0, rtol=1e-15)
    b2 = efpi.hammersley_b(idx, 2 ** 31)
    assert np.allclose(b2, np.mod(vdc + 0.5, 1.0) + 2.0 ** -33, atol=1e-15)


def test_inverse_normal_routine():
    from scipy.special import ndtri
    b = np.array([1e-9, 0.025, 0.3, 0.5, 0.975, 1 - 1e-7])
    assert np.allclose(ndtr(ndtri(b)), b, rtol=1e-12)
    assert ndtri(0.975) == pytest.approx(1.959963984540054, rel=1e-14)


def test_quiet_start_moments():
    n, ppc = 256, 400
    g = Grid(n, float(n))
    sch = efpi.Scheme(ppc=ppc, vth=0.3)
    nn, uu = synth.iaw_profile(n, float(n))
    cell, frac, v, w = efpi.load_particles(nn, uu, g, sch, synth.lift_shift(7))
    assert cell.size == n * ppc and np.all(np.diff(cell) >= 0)
    # weights reproduce the density: sum w = integral of the linear interpolant = L
    assert w.sum() == pytest.approx(float(n), rel=1e-12)
    # per-cell mean velocity ~ u and global thermal spread ~ vth (low-discrepancy error)
    x = efpi.particles_to_x(cell, frac, g)
    u_at = np.interp(x, np.arange(n + 1), np.append(uu, uu[0]))
    dv = v - u_at
    assert abs(np.mean(dv)) < 2e-3
    assert np.sqrt(np.mean(dv ** 2)) == pytest.approx(0.3, rel=5e-3)


def test_lift_block_correction_exact():
    n, lv = 128, 3
    g = Grid(n, float(n))
    sch = efpi.Scheme(levels=lv, ppc=50)
    coarse = synth.random_coarse(n >> lv, seed=9, levels=lv)
    cell, frac, v, w = efpi.lift(coarse, g, sch, synth.lift_shift(9))
    blk = cell >> lv
    scale = g.h * 2 ** (lv / 2)
    assert np.allclose(np.bincount(blk, weights=w), coarse[0] * scale, rtol=1e-12)
    assert np.allclose(np.bincount(blk, weights=w * v), coarse[1] * scale, rtol=1e-10, atol=1e-12)


def test_lift_then_restrict_close_to_identity():
    n, lv = 256, 4
    g = Grid(n, float(n))
    sch = efpi.Scheme(levels=lv, ppc=200)
    coarse = synth.random_coarse(n >> lv, seed=11, levels=lv)
    cell, frac, v, w = efpi.lift(coarse, g, sch, synth.lift_shift(11))
    x = efpi.particles_to_x(cell, frac, g)
    back = efpi.restrict_state(x, v, w, np.ones(x.size, bool), g, sch)
    assert metrics.rel_l2(back[0], coarse[0]) < 1e-3
    assert metrics.rel_l2(back[1], coarse[1]) < 1e-2


def test_piecewise_constant_lift_profile_inverts_restriction():
    n, lv = 64, 3
    g = Grid(n, float(n))
    sch = efpi.Scheme(levels=lv, lift_linear=False)
    coarse = synth.random_coarse(n >> lv, seed=12, levels=lv)
    nf, jf = efpi.lift_profile(coarse, g, sch)
    s, _ = efpi.haar_analysis(nf, lv)
    assert np.allclose(s, coarse[0], atol=1e-13)


def test_lift_deterministic_and_shift_sensitive():
    g = Grid(64, 64.0)
    sch = efpi.Scheme(levels=2, ppc=20)
    coarse = synth.random_coarse(16, seed=13, levels=2)
    a = efpi.lift(coarse, g, sch, 12345)
    b = efpi.lift(coarse, g, sch, 12345)
    c = efpi.lift(coarse, g, sch, 999)
    assert all(np.array_equal(p, q) for p, q in zip(a, b))
    assert not np.array_equal(a[2], c[2])


# ------------------------------------------------------------ end to end ----

def test_leap_zero_equals_pic():
    # Delta t = N_e dt: the projection adds nothing, and the last snapshot is the
    # plain restriction of the PIC state after N_e steps (tau_{N_e} = 0).
    n = 64
    g = Grid(n, float(n))
    sch = efpi.Scheme(levels=2, burst_steps=5, macro_dt=0.5, ppc=40)
    nn, uu = synth.iaw_profile(n, float(n))
    cell, frac, v, w = efpi.load_particles(nn, uu, g, sch, synth.lift_shift(14))
    x = efpi.particles_to_x(cell, frac, g)
    snaps, *_ = efpi.pic_burst(x, v, w, g, sch)
    nxt = efpi.project(snaps, g.dt, sch.macro_dt)
    xp, vh, al, phi = pic.pic_run(x, v, w, g, 5)
    vi = vh + 0.5 * g.dt * pic.gather(pic.field(phi, g), xp, g)
    ref = efpi.restrict_state(xp, vi, w, al, g, sch)
    assert np.allclose(nxt, ref, atol=1e-11)


@pytest.mark.slow
def test_efpi_error_grows_with_macro_step():
    # Parity unpinned beyond this trend: the projective error against full PIC
    # shrinks as Delta t approaches N_e dt (convergence claim of Sec. 4.1).
    n = 128
    g = Grid(n, float(n))
    nn, uu = synth.iaw_profile(n, float(n))
    errs = []
    for mdt in (2.0, 6.0, 12.0):
        sch = efpi.Scheme(levels=3, burst_steps=10, macro_dt=mdt, ppc=100)
        cell, frac, v, w = efpi.load_particles(nn, uu, g, sch, synth.lift_shift(15))
        x = efpi.particles_to_x(cell, frac, g)
        c0 = efpi.restrict_state(x, v, w, np.ones(x.size, bool), g, sch)
        nxt, _, _ = efpi.macro_step(c0, g, sch, synth.lift_shift(16))
        steps = int(round(mdt / g.dt))
        xp, vh, al, phi = pic.pic_run(x, v, w, g, steps)
        ref = efpi.restrict_state(xp, vh, w, al, g, sch)
        errs.append(metrics.rel_l2(nxt[0], ref[0]))
    assert errs[0] < errs[2]


def test_ensemble_mean():
    a, b, c = (np.full((2, 4), v) for v in (1.0, 2.0, 6.0))
    assert np.allclose(efpi.ensemble_mean([a, b, c]), 3.0)


def test_rel_l2_metric():
    assert metrics.rel_l2([1, 2], [1, 2]) == 0.0
    assert metrics.rel_l2([1, 0], [0, 1]) == pytest.approx(1.0)
    assert metrics.rel_l2([2.0], [1.0]) == pytest.approx(np.sqrt(1 / 5))


# ----------------------------------------------------- in-cell interpolation --
# Hand-worked quiet starts (App. C: density and mean velocity are interpolated
# linearly between the two nodes of a cell).  Node values n = (1, 3, 2, 5),
# u = (0.1, -0.2, 0.4, 0.0), h = 2, two ions per cell at offsets 1/4 and 3/4, cold
# ions (vth = 0) so that v = u(X) exactly; w = n(X) h / ppc = n(X).

HAND_N = np.array([1.0, 3.0, 2.0, 5.0])
HAND_U = np.array([0.1, -0.2, 0.4, 0.0])


def test_load_particles_interpolates_n_and_u_in_the_cell_periodic():
    g = Grid(4, 8.0)
    sch = efpi.Scheme(ppc=2, vth=0.0)
    cell, frac, v, w = efpi.load_particles(HAND_N, HAND_U, g, sch, 12345)
    assert list(cell) == [0, 0, 1, 1, 2, 2, 3, 3]
    assert list(frac) == [0.25, 0.75] * 4
    # cell 3 takes its right node from node 0 (periodic)
    assert np.allclose(w, [1.5, 2.5, 2.75, 2.25, 2.75, 4.25, 4.0, 2.0], rtol=0, atol=1e-15)
    assert np.allclose(v, [0.025, -0.125, -0.05, 0.25, 0.3, 0.1, 0.025, 0.075], rtol=0,
                       atol=1e-15)


def test_load_particles_interpolates_n_and_u_in_the_cell_walls():
    g = Grid(4, 8.0, bc=WALLS)
    sch = efpi.Scheme(ppc=2, vth=0.0)
    n5 = np.append(HAND_N, 3.0)            # wall node 4
    u5 = np.append(HAND_U, -0.4)
    cell, frac, v, w = efpi.load_particles(n5, u5, g, sch, 12345)
    assert np.allclose(w[6:], [4.5, 3.5], rtol=0, atol=1e-15)        # (5, 3) at 1/4, 3/4
    assert np.allclose(v[6:], [-0.1, -0.3], rtol=0, atol=1e-15)      # (0, -0.4)
    assert np.allclose(w[:6], [1.5, 2.5, 2.75, 2.25, 2.75, 4.25], rtol=0, atol=1e-15)


def test_lift_profile_linear_between_block_centres():
    # 8 cells, blocks of 4 (l = 2) with means 1 and 3 (coefficients 2^{l/2} times
    # the means); centres at 1.5 and 5.5.  Periodic: node 0 lies 2.5 to the right
    # of the previous period's centre 5.5 - 8, a fraction 0.625 of the way to 1.5.
    sch = efpi.Scheme(levels=2, lift_linear=True)
    coarse = np.array([[2.0, 6.0], [0.4, -0.2]])           # means (1, 3) and (0.2, -0.1)
    n, j = efpi.lift_profile(coarse, Grid(8, 8.0), sch)
    assert np.allclose(n, [1.75, 1.25, 1.25, 1.75, 2.25, 2.75, 2.75, 2.25], rtol=0, atol=1e-15)
    assert np.allclose(j, [0.0875, 0.1625, 0.1625, 0.0875, 0.0125, -0.0625, -0.0625, 0.0125],
                       rtol=0, atol=1e-15)
    # walls: constant beyond the end centres, node 8 included
    n, _ = efpi.lift_profile(coarse, Grid(8, 8.0, bc=WALLS), sch)
    assert np.allclose(n, [1.0, 1.0, 1.25, 1.75, 2.25, 2.75, 3.0, 3.0, 3.0], rtol=0, atol=1e-15)
    # and the piecewise-constant inverse Haar without the flag
    n, _ = efpi.lift_profile(coarse, Grid(8, 8.0), efpi.Scheme(levels=2, lift_linear=False))
    assert np.allclose(n, [1.0] * 4 + [3.0] * 4, rtol=0, atol=1e-15)


# ---------------------------------------------------- EFREE second moment ---

def _efree_coarse(nc, levels, seed):
    """Three coarse moments of positive density and temperature."""
    return synth.random_coarse_efree(nc, seed=seed, levels=levels)


def test_second_moment_restriction_by_hand():
    # tau = 0, l = 0: node charge / h with CIC; two ions in an 8-cell periodic grid
    g = Grid(8, 8.0)
    x = np.array([1.25, 6.5])
    v = np.array([2.0, -1.0])
    w = np.array([0.5, 2.0])
    out = efpi.restrict_snapshot(x, v, np.zeros(2), w, 0.0, g, 0, False, moments=3)
    assert out.shape == (3, 8)
    want_s = np.zeros(8)
    want_s[1], want_s[2] = 0.75 * 0.5 * 4.0, 0.25 * 0.5 * 4.0     # w v^2 = 2 split 3/4, 1/4
    want_s[6], want_s[7] = 0.5 * 2.0, 0.5 * 2.0                   # w v^2 = 2 split in half
    assert np.allclose(out[2], want_s, rtol=0, atol=1e-15)
    # the first two rows are the two-moment restriction
    assert np.array_equal(out[:2], efpi.restrict_snapshot(x, v, np.zeros(2), w, 0.0, g, 0, False))


def test_coevolving_moments_by_hand():
    # App. B with tau = 2 and a stored field: X~ = X + tau V, V~ = V + tau E_n(X); the
    # mass, w V~ and w V~^2 go by CIC to the nodes around X~ (l = 0, h = 1)
    g = Grid(8, 8.0)
    x = np.array([1.25, 6.5])
    v = np.array([0.5, -0.25])
    e = np.array([0.1, -0.2])
    w = np.array([0.5, 2.0])
    out = efpi.restrict_snapshot(x, v, e, w, 2.0, g, 0, True, moments=3)
    # X~ = 2.25 (3/4 to node 2, 1/4 to node 3) and 6.0 (all to node 6); V~ = 0.7, -0.65
    want = np.zeros((3, 8))
    for m, (a, b) in enumerate(((0.5, 2.0), (0.5 * 0.7, 2.0 * -0.65),
                                (0.5 * 0.49, 2.0 * 0.4225))):
        want[m, 2], want[m, 3], want[m, 6] = 0.75 * a, 0.25 * a, b
    assert np.allclose(out, want, rtol=0, atol=1e-14)


def test_temperature_profile_by_hand():
    sch = efpi.Scheme(n_floor=1e-3)
    n = np.array([2.0, 1.0, 1e-4, 4.0])
    j = np.array([1.0, 0.5, 0.0, -2.0])
    s = np.array([2.5, 0.2, 1.0, 1.0])
    # T = s/n - (j/n)^2: 1.25 - 0.25; 0.2 - 0.25 < 0 -> 0; below the floor -> 0; 0.25 - 0.25
    assert np.allclose(efpi.temperature_profile(n, j, s, sch), [1.0, 0.0, 0.0, 0.0], atol=1e-15)


def test_load_particles_with_a_temperature_profile_by_hand():
    from scipy.special import ndtri
    g = Grid(4, 8.0)
    sch = efpi.Scheme(ppc=2, vth=123.0)        # vth is not used with a temperature profile
    t = np.array([0.04, 0.36, 1.0, 0.16])
    shift = 12345
    cell, frac, v, w = efpi.load_particles(HAND_N, HAND_U, g, sch, shift, t)
    b = efpi.hammersley_b(np.arange(8, dtype=np.uint64), shift)
    # T linear in the cell (cell 3 takes node 0 on the right), sigma = sqrt(T)
    t_at = [0.12, 0.28, 0.52, 0.84, 0.79, 0.37, 0.13, 0.07]
    u_at = [0.025, -0.125, -0.05, 0.25, 0.3, 0.1, 0.025, 0.075]
    assert np.allclose(v, np.array(u_at) + np.sqrt(t_at) * ndtri(b), rtol=0, atol=1e-14)


def test_efree_block_correction_exact():
    n, lv = 128, 3
    g = Grid(n, float(n))
    sch = efpi.Scheme(levels=lv, ppc=50, moments=3)
    coarse, _ = _efree_coarse(n >> lv, lv, 19)
    cell, frac, v, w = efpi.lift(coarse, g, sch, synth.lift_shift(19))
    blk = cell >> lv
    scale = g.h * 2 ** (lv / 2)
    assert np.allclose(np.bincount(blk, weights=w), coarse[0] * scale, rtol=1e-12)
    assert np.allclose(np.bincount(blk, weights=w * v), coarse[1] * scale, rtol=1e-10, atol=1e-12)
    assert np.allclose(np.bincount(blk, weights=w * v * v), coarse[2] * scale, rtol=1e-10)


def test_efree_lift_carries_the_block_temperature():
    # a uniform plasma at rest with a temperature that differs from vth^2: the loaded
    # spread follows the coarse second moment, not vth
    n, lv, ppc = 256, 4, 400
    g = Grid(n, float(n))
    sch = efpi.Scheme(levels=lv, ppc=ppc, moments=3, vth=0.3)
    nc = n >> lv
    scale = 2.0 ** (lv / 2)
    coarse = np.stack([np.full(nc, scale), np.full(nc, 0.2 * scale),
                       np.full(nc, (0.04 + 0.5) * scale)])       # u = 0.2, T = 0.5
    cell, frac, v, w = efpi.lift(coarse, g, sch, synth.lift_shift(3), correct=False)
    assert np.mean(v) == pytest.approx(0.2, abs=2e-3)
    assert np.sqrt(np.mean((v - 0.2) ** 2)) == pytest.approx(np.sqrt(0.5), rel=5e-3)
    x = efpi.particles_to_x(cell, frac, g)
    back = efpi.restrict_state(x, v, w, np.ones(x.size, bool), g, sch)
    assert metrics.rel_l2(back[2], coarse[2]) < 2e-3


def test_efree_snapshots_equal_in_free_streaming():
    # App. B with E = 0 for the second moment too: V~ = V, so w V~^2 moves with X~
    g = Grid(64, 64.0, closure=NOFIELD)
    sch = efpi.Scheme(levels=2, burst_steps=6, macro_dt=3.0, ppc=32, moments=3)
    nn, uu = synth.iaw_profile(64, 64.0)
    cell, frac, v, w = efpi.load_particles(nn, uu, g, sch, synth.lift_shift(5))
    snaps, *_ = efpi.pic_burst(efpi.particles_to_x(cell, frac, g), v, w, g, sch)
    assert snaps.shape[1] == 3
    assert np.max(np.abs(snaps - snaps[0])) < 1e-10
