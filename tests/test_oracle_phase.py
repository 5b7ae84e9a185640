"""Pins of the phase-space coarse-variable oracle (Sec. 3.3, App. A, App. C).

Each check uses a property fixed by the mathematics: the Coiflet conditions
themselves and the vanishing moments of the scaling function and wavelet
measured on the functions (cascade), perfect reconstruction and Parseval for the
periodized transform,
preservation of the first four moments by the scaling coefficients, mass
conservation of the full-weighting restriction, exact interpolation of linear
data, the histogram's mass, and the repaired CDF's monotonicity and
conservation of M_0 and M_1 (the lemma of App. C).
"""
import numpy as np
import pytest

import phase_cases
from oracle import phase
from oracle.phase import PhaseScheme
from oracle.pic import Grid
from phase_cases import LIFT_CASES


@pytest.fixture(scope="module")
def h():
    return phase.coiflet_filter()


@pytest.fixture(scope="module")
def product_taps():
    from paper_1610_01071_amd.phase import coiflet_taps
    return {12: coiflet_taps(12), 6: coiflet_taps(6)}


def test_coiflet_conditions(h):
    assert h.size == 12
    assert np.max(np.abs(phase.coiflet_conditions(h))) < 1e-12
    g = phase.highpass(h)
    assert abs(np.dot(h, g)) < 1e-14                      # low and high pass orthogonal
    k = np.arange(12, dtype=float)
    assert max(abs(np.sum(g * k ** p)) for p in range(4)) < 1e-10


def _point_values(h, levels):
    """phi at i 2^-levels on [0, L-1], computed here apart from the oracle: the
    integer values by power iteration of the refinement map (not an eigensolver),
    then the two-scale relation phi(y) = sqrt 2 sum_k h_k phi(2y - k) per level."""
    h = np.asarray(h, dtype=np.float64)
    n = h.size
    vals = np.ones(n) / n
    for _ in range(3000):
        nxt = np.array([sum(np.sqrt(2.0) * h[2 * i - m] * vals[m] for m in range(n)
                            if 0 <= 2 * i - m < n) for i in range(n)])
        vals = nxt / nxt.sum()
    for j in range(levels):
        step = 1 << j
        size = (n - 1) * 2 * step + 1
        nxt = np.zeros(size)
        for k in range(n):
            src = np.arange(size) - k * step
            ok = (src >= 0) & (src < vals.size)
            nxt[ok] += np.sqrt(2.0) * h[k] * vals[src[ok]]
        vals = nxt
    return vals


def _cascade_moments(h, origin, order, levels=12):
    """Moments of phi about `origin` (orders 0 .. order-1) and of psi (orders
    0 .. order-1), by the trapezoid rule on the dyadic point values (the end
    values are zero); psi(y) = sqrt 2 sum_k g_k phi(2y - k)."""
    n = len(h)
    phi = _point_values(h, levels)
    dy = 2.0 ** -levels
    y = np.arange(phi.size) * dy
    mphi = [np.sum(phi * (y - origin) ** p) * dy for p in range(order)]
    g = ((-1.0) ** np.arange(n)) * np.asarray(h)[::-1]
    yy = np.arange((n - 1) * 2 ** (levels - 1) + 1) * 2.0 * dy    # psi's grid: 2^-(levels-1)
    psi = np.zeros(yy.size)
    for k in range(n):
        src = 4 * np.arange(yy.size) - k * (1 << levels)
        ok = (src >= 0) & (src < phi.size)
        psi[ok] += np.sqrt(2.0) * g[k] * phi[src[ok]]
    mpsi = [np.sum(psi * yy ** p) * 2.0 * dy for p in range(order)]
    return mphi, mpsi


@pytest.mark.parametrize("which", ["oracle", "product12", "product6"])
def test_coiflet_moments_measured_on_the_scaling_function(which, h, product_taps):
    # App. A: psi has vanishing moments 0..2K-1 and phi vanishing moments 1..2K-1
    # about the origin of its support (tap 2K), measured on phi and psi themselves
    taps = {"oracle": h, "product12": product_taps[12], "product6": product_taps[6]}[which]
    order = len(taps) // 3
    mphi, mpsi = _cascade_moments(taps, origin=order, order=order)
    assert abs(mphi[0] - 1.0) < 1e-12
    assert max(abs(m) for m in mphi[1:]) < 1e-10
    assert max(abs(m) for m in mpsi) < 1e-10


def test_scaling_function_matches_the_refinement_relation(h):
    assert np.max(np.abs(phase.scaling_function(h, 10) - _point_values(h, 10))) < 1e-12


def test_product_and_oracle_coiflets_agree(h, product_taps):
    # two derivations that share no code (lattice angles and Levenberg-Marquardt in
    # the library, least squares over the taps and a cascade symmetry test here)
    # select the same filter
    assert np.max(np.abs(product_taps[12] - h)) < 1e-10
    assert np.max(np.abs(phase.coiflet_conditions(product_taps[12]))) < 1e-12


def test_dwt_perfect_reconstruction_and_parseval(h):
    x = np.random.default_rng(1).standard_normal((4, 128))
    a, d = phase.dwt_level(x, h)
    assert np.max(np.abs(phase.idwt_level(a, d, h) - x)) < 1e-13
    assert np.allclose(np.sum(x * x, axis=-1), np.sum(a * a, axis=-1) + np.sum(d * d, axis=-1),
                       rtol=1e-13)


def test_scaling_coefficients_keep_the_first_four_moments(h):
    # A sharp column well inside the periodic window: dropping the details of
    # three levels leaves its moments of order 0..3 unchanged (four vanishing
    # moments of the wavelet), while order 4 changes.
    n = 256
    k = np.arange(n, dtype=float)
    x = np.exp(-0.5 * ((k - 128.0) / 2.5) ** 2) + 0.5 * (np.abs(k - 110.0) < 3.0)
    y = phase.from_scaling_coefficients(phase.scaling_coefficients(x, h, 3), h, 3)
    mom = lambda z, p: np.sum(z * k ** p)
    for p in range(4):
        assert abs(mom(y, p) - mom(x, p)) < 1e-9 * abs(mom(x, p)) + 1e-9
    assert abs(mom(y, 4) - mom(x, 4)) > 1e-8 * abs(mom(x, 4))


def test_full_weighting_and_interpolation():
    f = np.random.default_rng(2).uniform(0.5, 1.5, (64, 3))
    c = phase.full_weighting(f)
    assert np.allclose(2.0 * c.sum(axis=0), f.sum(axis=0), rtol=1e-14)   # spacing doubles
    const = np.full((16, 2), 0.7)
    assert np.array_equal(phase.midpoint_interpolation(const), np.full((32, 2), 0.7))
    lin = np.arange(16, dtype=float)[:, None] * np.ones((1, 2))
    fine = phase.midpoint_interpolation(lin)
    assert np.allclose(fine[:-1], (np.arange(31) / 2.0)[:, None])        # interior: linear
    # restriction of the interpolant of a constant is that constant
    assert np.allclose(phase.full_weighting(phase.midpoint_interpolation(const)), const)


def test_histogram_mass_and_momentum(h):
    g = Grid(32, 32.0)
    ps = PhaseScheme(v_min=-2.0, v_max=2.0, jf=6)
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 32, 5000)
    v = rng.uniform(-1.9, 1.9, 5000)
    w = rng.uniform(0.5, 1.5, 5000) / 100
    f = phase.phase_histogram(x, v, w, g, ps)
    assert np.sum(f) * g.h * ps.dv == pytest.approx(np.sum(w), rel=1e-13)
    centres = ps.v_min + (np.arange(ps.n_vf) + 0.5) * ps.dv
    kv = np.floor((v - ps.v_min) / ps.dv).astype(int)
    assert np.sum(f * centres[None, :]) * g.h * ps.dv == \
        pytest.approx(np.sum(w * centres[kv]), rel=1e-12)
    # coarsening conserves mass: one coarse node stands for 2^l fine ones, and the
    # column's scaling coefficients sum to 2^{(J_f - J_c)/2} times the fine ones
    ps2 = PhaseScheme(levels=2, v_min=-2.0, v_max=2.0, jf=6, jc=4)
    c = phase.coarsen(f, ps2, h)
    mass = np.sum(c) * 2 ** ((ps2.jf - ps2.jc) / 2.0) * 2 ** (ps2.jf / 2.0) / (4.0) \
        * (4 * g.h) * ps2.dv
    assert mass == pytest.approx(np.sum(w), rel=1e-12)


def _bad_cdf(seed, n=64, noise=0.08):
    rng = np.random.default_rng(seed)
    dens = np.exp(-0.5 * ((np.arange(n) - 30.0) / 6.0) ** 2) + noise * rng.standard_normal(n)
    dens[:3] = -0.05                       # a negative edge
    F = np.concatenate([[0.0], np.cumsum(dens)])
    return F / F[-1]


@pytest.mark.parametrize("seed", range(6))
def test_repaired_cdf_is_monotone_and_keeps_m0_m1(seed):
    F = _bad_cdf(seed)
    assert np.any(np.diff(F) < 0) or np.any(F < 0)
    R = phase.repair_cdf(F)
    assert R[0] == 0.0 and R[-1] == 1.0
    assert np.all(np.diff(R) >= -1e-15) and np.all(R >= -1e-15) and np.all(R <= 1 + 1e-15)
    # M_1 = n - sum_{k<n} F[k] (M_0 = 1 by construction): kept by every ramp
    assert np.sum(R) == pytest.approx(np.sum(F), rel=1e-12, abs=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_repair_is_monotone_under_heavy_noise(seed):
    # large oscillations can leave no momentum-conserving ramp below F[n] (the
    # paper's pathological case); the result is still a valid CDF
    R = phase.repair_cdf(_bad_cdf(seed, noise=0.3))
    assert R[0] == 0.0 and R[-1] == 1.0 and np.all(np.diff(R) >= -1e-15)


def test_repair_keeps_a_monotone_cdf():
    F = np.concatenate([[0.0], np.cumsum(np.linspace(0.1, 1.0, 40))])
    F /= F[-1]
    assert np.max(np.abs(phase.repair_cdf(F) - F)) < 1e-15   # up to the reflection's rounding


def test_repair_of_a_single_dip_by_hand():
    # F = [0, .3, .2, .6, 1]: one drop after index 1.  k0 = 1, k1 = 3, k+ = 2,
    # k- = 0; slope 2/(2-0-1) * ((0 + .3)/2 - 0) = .3 fits under F[2] = .2? no:
    # 0 + 1 * .3 > .2, so k+ = 3: slope 2/2 * ((0 + .3 + .2)/3 - 0) = 1/6, F[1] = 1/6,
    # F[2] = 1/3 <= .6.  The backward pass gives the same here.
    F = np.array([0.0, 0.3, 0.2, 0.6, 1.0])
    fwd = phase._interior_forward(F)
    assert np.allclose(fwd, [0.0, 1 / 6, 1 / 3, 0.6, 1.0])
    assert np.sum(fwd) == pytest.approx(np.sum(F))


def test_inverse_cdf_of_a_uniform_column():
    ps = PhaseScheme(v_min=-1.0, v_max=3.0, jf=5)
    F = np.arange(ps.n_vf + 1) / ps.n_vf
    b = np.linspace(0.01, 0.99, 17)
    assert np.allclose(phase.inverse_cdf(F, b, ps), ps.v_min + b * (ps.v_max - ps.v_min))


def test_lift_restores_density_and_mean_velocity(h):
    # A drifting Maxwellian column everywhere, coarsened and lifted: the loaded ions
    # carry the density and mean velocity (quiet start, so to sampling accuracy).
    g = Grid(64, 64.0)
    ps = PhaseScheme(levels=2, v_min=-2.0, v_max=2.0, jf=7, jc=5, ppc=400)
    centres = ps.v_min + (np.arange(ps.n_vf) + 0.5) * ps.dv
    col = np.exp(-0.5 * ((centres - 0.3) / 0.32) ** 2)
    col /= np.sum(col) * ps.dv
    f = np.tile(col, (64, 1))
    cell, frac, v, w = phase.lift_phase(phase.coarsen(f, ps, h), g, ps, h, 12345)
    assert np.sum(w) == pytest.approx(64.0, rel=1e-3)
    assert np.sum(w * v) / np.sum(w) == pytest.approx(0.3, abs=2e-3)
    assert np.sqrt(np.sum(w * (v - 0.3) ** 2) / np.sum(w)) == pytest.approx(0.32, rel=2e-2)


def test_free_streaming_burst_snapshots_are_the_state_at_t_plus_dt(h):
    # Without a field the co-evolving map X + (Dt - p dt) v sends every snapshot to
    # the particles advanced by the whole macro step, so all snapshots agree and
    # equal the restriction of x + Dt v (the exactness of App. B for free streaming).
    from oracle.pic import NOFIELD
    g = Grid(32, 32.0, closure=NOFIELD, dt=0.1)
    ps = PhaseScheme(levels=1, v_min=-2.0, v_max=2.0, jf=6, jc=4, burst_steps=5, macro_dt=2.0)
    rng = np.random.default_rng(4)
    x = rng.uniform(0, 32, 4000)
    v = rng.uniform(-1.5, 1.5, 4000)
    w = np.full(4000, 0.01)
    snaps = phase.phase_burst(x, v, w, g, ps, h)
    want = phase.coarsen(phase.phase_histogram(np.mod(x + ps.macro_dt * v, 32.0), v, w, g, ps),
                         ps, h)
    for p in range(ps.burst_steps + 1):
        assert np.max(np.abs(snaps[p] - want)) < 1e-10 * np.max(np.abs(want))


def test_fixed_point_restricted_histogram_equals_full_weighting_of_the_histogram(h):
    # the integer form with the composed hat weights is l levels of eq. 3.8 applied
    # to the CIC x NGP histogram, up to the 2^-40 quantisation of the charge
    g = Grid(64, 64.0)
    ps = PhaseScheme(levels=3, v_min=-2.0, v_max=2.0, jf=6, jc=4)
    rng = np.random.default_rng(8)
    n = 20000
    cell = rng.integers(0, 64, n).astype(np.int16)
    frac = rng.random(n, dtype=np.float32)
    v = rng.uniform(-2.2, 2.2, n).astype(np.float32)
    w = (rng.uniform(0.5, 1.5, n) / 300).astype(np.float32)
    H = phase.restricted_histogram_fx(cell, frac, v, w, 64, ps)
    x = (cell.astype(np.float64) + frac.astype(np.float64)) * g.h
    f = phase.phase_histogram(x, v.astype(np.float64), w.astype(np.float64), g, ps)
    for _ in range(ps.levels):
        f = phase.full_weighting(f)
    dens = H.astype(np.float64) / 2.0 ** 40 / (4.0 ** ps.levels * g.h * ps.dv)
    assert np.max(np.abs(dens - f)) < 1e-9 * np.max(np.abs(f))
    c = phase.coarse_from_histogram_fx(H, ps, g.h, h)
    assert np.max(np.abs(c - phase.coarsen(phase.phase_histogram(
        x, v.astype(np.float64), w.astype(np.float64), g, ps), ps, h))) < 1e-9 * np.max(np.abs(c))




@pytest.mark.parametrize("n,levels,jf,jc,ppc,filt", LIFT_CASES)
def test_repair_sum_order_does_not_decide_the_gpu_cases(n, levels, jf, jc, ppc, filt,
                                                        monkeypatch):
    # The repair's sums run in index order (its decisions compare them).  With
    # pairwise sums instead, every lift case of the GPU parity tests gives the
    # same ions: no decision there rests on the summation order.
    ps = PhaseScheme(levels=levels, v_min=-2.0, v_max=2.0, jf=jf, jc=jc, ppc=ppc)
    hh = phase_cases.taps(filt)
    coarse = phase_cases.phase_state(n, 50, 3, ps, hh)
    g = Grid(n, float(n))
    a = phase.lift_phase(coarse, g, ps, hh, 4242)
    monkeypatch.setattr(phase, "_seqsum", lambda x: float(np.sum(np.asarray(x, np.float64))))
    b = phase.lift_phase(coarse, g, ps, hh, 4242)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for k in (2, 3):
        assert np.max(np.abs(a[k] - b[k])) <= 1e-12 * np.max(np.abs(a[k]))


def _bitrev32(i):
    return int(format(i, "032b")[::-1], 2)


def test_lift_phase_interpolates_between_the_two_nodes(monkeypatch):
    # Hand-worked lift (App. C: values at a particle are interpolated linearly
    # between the two closest grid points).  Two periodic cells, h = 1, 16 bins of
    # dv = 1/4 over [-2, 2).  Node 0 holds density 4 in bin 5 only (n = 1), node 1
    # density 8 in bin 9 only (n = 2); both CDFs are valid, so the repair keeps them
    # and a node's inverse CDF at b is v_min + (bin + b) dv.  Two ions per cell.
    ps = PhaseScheme(levels=0, v_min=-2.0, v_max=2.0, jf=4, jc=4, ppc=2)
    fine = np.zeros((2, 16))
    fine[0, 5] = 4.0
    fine[1, 9] = 8.0
    monkeypatch.setattr(phase, "refine", lambda coarse, ps_, h_: fine)
    shift = 987654321
    cell, frac, v, w = phase.lift_phase(None, Grid(2, 2.0), ps, None, shift)
    assert list(cell) == [0, 0, 1, 1] and list(frac) == [0.25, 0.75, 0.25, 0.75]
    b = [((_bitrev32(i) + shift) % 2 ** 32 + 0.5) / 2.0 ** 32 for i in range(4)]
    # cell 0: bin 5 -> 9 across the cell, i.e. 5 + 4 frac; cell 1: 9 -> 5
    expect_v = [-2.0 + 0.25 * (5 + 1 + b[0]), -2.0 + 0.25 * (5 + 3 + b[1]),
                -2.0 + 0.25 * (9 - 1 + b[2]), -2.0 + 0.25 * (9 - 3 + b[3])]
    assert np.allclose(v, expect_v, rtol=0, atol=1e-14)
    # w = n(X) h / ppc with n = 1 at node 0 and 2 at node 1
    assert np.allclose(w, [0.625, 0.875, 0.875, 0.625], rtol=0, atol=1e-15)
